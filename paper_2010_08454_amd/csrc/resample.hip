// resample.hip -- FP64 log-sum-exp / ESS normaliser, integer-rule systematic
// resampling, resampling fused with the gather of structure-of-arrays state,
// and the raw Philox stream entry.
//
// The normaliser is the weight normalisation of importance sampling (paper
// Sec. 3.6.2); resampling between factors is the particle-based inference the
// paper names as future work (Sec. 6).  Resampling quantises the weights to
// integers (q_i = floor(exp(lw_i - max) 2^k)) so that the prefix sum, and with
// it every ancestor index, is exact and independent of the reduction order.
#include "device.h"
#include "host.h"
#include "kernels.h"
#include "timing.h"

namespace ppl {

constexpr int kRedThreads = 256;
constexpr int kRedBlocksMax = 1024;
constexpr int kScanItems = 8;                          // items per thread in the scan
constexpr int kScanTile = kRedThreads * kScanItems;    // items per block
constexpr int kGatherPer = 4;                          // outputs per thread of the gather
constexpr int kGatherOut = kRedThreads * kGatherPer;   // outputs per gather workgroup
constexpr int kGatherStage = 2 * kGatherOut;           // staged prefix sums per workgroup

// -------------------------------------------------------- normaliser ----
template <typename T>
__global__ __launch_bounds__(kRedThreads) void lse_partial_kernel(const T *__restrict__ lw, int64_t n,
                                                                  double *__restrict__ part) {
    Partial<0> p = partial_empty<0>();
    const int64_t stride = (int64_t)gridDim.x * kRedThreads;
    double m = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
        const double v = (double)lw[i];
        if (isnan(v)) p.nan += 1.0;
        else if (v > m) m = v;
    }
    p.m = m;
    if (m > -INFINITY) {
        for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
            const double v = (double)lw[i];
            if (!isnan(v)) {
                const double e = exp(v - m);
                p.s1 += e;
                p.s2 += e * e;
            }
        }
    }
    partial_block_reduce_store<0, kRedThreads / 64>(p, part + (size_t)blockIdx.x * 4);
}

__global__ __launch_bounds__(kRedThreads) void lse_finalize_kernel(const double *__restrict__ part, int nb,
                                                                   double *__restrict__ out) {
    __shared__ double rec[4];
    records_block_reduce_store<0, kRedThreads / 64>(part, 0, nb, rec);
    __syncthreads();
    if (threadIdx.x) return;
    const Partial<0> a = partial_load<0>(rec);
    if (a.nan > 0) {
        for (int k = 0; k < 5; ++k) out[k] = NAN;
    } else if (!(a.m > -INFINITY)) {
        out[0] = -INFINITY; out[1] = 0.0; out[2] = 0.0; out[3] = -INFINITY; out[4] = 0.0;
    } else {
        out[0] = a.m; out[1] = a.s1; out[2] = a.s2; out[3] = a.m + log(a.s1); out[4] = a.s1 * a.s1 / a.s2;
    }
}

static int64_t red_blocks(int64_t n) {
    int64_t b = (n + kRedThreads - 1) / kRedThreads;
    return b < 1 ? 1 : (b > kRedBlocksMax ? kRedBlocksMax : b);
}

size_t lse_ws_bytes(int64_t n) { return (size_t)red_blocks(n) * 4 * sizeof(double); }

int run_lse(const void *lw, bool f64, int64_t n, double *out5, void *ws, hipStream_t st) {
    const int64_t nb = red_blocks(n);
    double *part = (double *)ws;
    if (f64)
        hipLaunchKernelGGL(lse_partial_kernel<double>, dim3((unsigned)nb), dim3(kRedThreads), 0, st,
                           (const double *)lw, n, part);
    else
        hipLaunchKernelGGL(lse_partial_kernel<float>, dim3((unsigned)nb), dim3(kRedThreads), 0, st,
                           (const float *)lw, n, part);
    PPL_LAUNCH_CHECK("lse_partial_kernel");
    hipLaunchKernelGGL(lse_finalize_kernel, dim3(1), dim3(kRedThreads), 0, st, part, (int)nb, out5);
    PPL_LAUNCH_CHECK("lse_finalize_kernel");
    return PPL_OK;
}

// -------------------------------------------------------- resampling ----
// Workspace layout (all 256-byte aligned):
//   blockmax [nb] double | total [nb] u64 | prefix [nb] u64 | meta [4] u64 |
//   ends [ng + 1] i64 | qloc [n] u64
struct ResampleWs {
    double *blockmax;
    uint64_t *total, *prefix, *meta, *qloc;
    int64_t *ends;
};

static int64_t scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }
static int64_t gather_blocks(int64_t n) { return (n + kGatherOut - 1) / kGatherOut; }

static ResampleWs resample_layout(void *ws, int64_t n) {
    const int64_t nb = scan_blocks(n);
    char *p = (char *)ws;
    ResampleWs r;
    r.blockmax = (double *)p; p += align_up(nb * sizeof(double), 256);
    r.total = (uint64_t *)p; p += align_up(nb * sizeof(uint64_t), 256);
    r.prefix = (uint64_t *)p; p += align_up(nb * sizeof(uint64_t), 256);
    r.meta = (uint64_t *)p; p += 256;
    r.ends = (int64_t *)p; p += align_up((gather_blocks(n) + 1) * sizeof(int64_t), 256);
    r.qloc = (uint64_t *)p;
    return r;
}

size_t resample_ws_bytes(int64_t n) {
    const int64_t nb = scan_blocks(n);
    return align_up(nb * sizeof(double), 256) + 2 * align_up(nb * sizeof(uint64_t), 256) + 256 +
           align_up((gather_blocks(n) + 1) * sizeof(int64_t), 256) + align_up(n * sizeof(uint64_t), 256);
}

__host__ __device__ inline int quant_bits(int64_t n) {
    int c = 0;
    while (((int64_t)1 << c) < n) ++c;
    return 62 - c;
}

// Exact partial maxima of the log-weights, one per block of a grid of at most
// kRedBlocksMax blocks (NaN entries are ignored here; run_resample rejects NaN
// through the normaliser's flag).
template <typename T>
__global__ __launch_bounds__(kRedThreads) void tile_max_kernel(const T *__restrict__ lw, int64_t n,
                                                               double *__restrict__ blockmax) {
    __shared__ double red[kRedThreads / 64];
    double m = -INFINITY;
    const int64_t stride = (int64_t)gridDim.x * kRedThreads;
    int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {   // four independent loads in flight
        const double v0 = lw[i], v1 = lw[i + stride], v2 = lw[i + 2 * stride], v3 = lw[i + 3 * stride];
        m = fmax(m, fmax(fmax(v0, v1), fmax(v2, v3)));
    }
    for (; i < n; i += stride) m = fmax(m, (double)lw[i]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = red[0];
        for (int w = 1; w < kRedThreads / 64; ++w) v = fmax(v, red[w]);
        blockmax[blockIdx.x] = v;
    }
}

__device__ __forceinline__ uint64_t wave_inclusive_scan_u64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Quantise and scan one tile: qloc[i] = inclusive sum of q within the tile,
// total[b] = tile sum.  Every block first reduces the nm partial maxima itself.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void quant_scan_kernel(const T *__restrict__ lw, int64_t n, int nm,
                                                                 const double *__restrict__ blockmax, int kbits,
                                                                 uint64_t *__restrict__ qloc,
                                                                 uint64_t *__restrict__ total) {
    __shared__ double smax[kRedThreads / 64];
    __shared__ uint64_t wsum[kRedThreads / 64];
    double m = -INFINITY;
    for (int b = threadIdx.x; b < nm; b += kRedThreads) m = fmax(m, blockmax[b]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = m;
    __syncthreads();
    m = smax[0];
#pragma unroll
    for (int w = 1; w < kRedThreads / 64; ++w) m = fmax(m, smax[w]);

    // Quantise with striped (coalesced) loads, then scan in blocked order: the
    // tile passes through LDS both ways so loads and stores stay coalesced.
    __shared__ uint64_t sbuf[kScanTile];
    const int64_t tile0 = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = tile0 + k * kRedThreads + threadIdx.x;
        uint64_t v = 0;
        if (i < n) {
            const double e = exp((double)lw[i] - m);
            if (e >= 0.0) v = (uint64_t)floor(ldexp(e, kbits));   // NaN entries carry no weight
        }
        sbuf[k * kRedThreads + threadIdx.x] = v;
    }
    __syncthreads();
    uint64_t q[kScanItems];
    uint64_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        run += sbuf[threadIdx.x * kScanItems + k];
        q[k] = run;
    }
    const uint64_t incl = wave_inclusive_scan_u64(run);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint64_t off = incl - run;
    for (int w = 0; w < wv; ++w) off += wsum[w];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) sbuf[threadIdx.x * kScanItems + k] = q[k] + off;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = tile0 + k * kRedThreads + threadIdx.x;
        if (i < n) qloc[i] = sbuf[k * kRedThreads + threadIdx.x];
    }
    if (threadIdx.x == kRedThreads - 1) total[blockIdx.x] = off + run;
}

// Exclusive prefix of the tile totals, S, and U = floor(R S / 2^64).  One
// workgroup: each thread sums a contiguous chunk of tiles, the chunk sums are
// scanned across the workgroup, and each thread writes its chunk's prefixes.
constexpr int kPrefixThreads = 1024;

__global__ __launch_bounds__(kPrefixThreads) void tile_prefix_kernel(const uint64_t *__restrict__ total, int nb,
                                                                     Key key, uint32_t step, uint32_t inst,
                                                                     uint64_t *__restrict__ prefix,
                                                                     uint64_t *__restrict__ meta) {
    __shared__ uint64_t wsum[kPrefixThreads / 64];
    const int per = (nb + kPrefixThreads - 1) / kPrefixThreads;
    const int b0 = threadIdx.x * per;
    const int b1 = b0 + per < nb ? b0 + per : nb;
    // chunk loads in batches of eight independent loads
    uint64_t sum = 0;
    for (int b = b0; b < b1; b += 8) {
        uint64_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = b + k < b1 ? total[b + k] : 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += v[k];
    }
    const uint64_t incl = wave_inclusive_scan_u64(sum);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint64_t off = incl - sum;
    for (int w = 0; w < wv; ++w) off += wsum[w];
    for (int b = b0; b < b1; b += 8) {
        uint64_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = b + k < b1 ? total[b + k] : 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (b + k < b1) prefix[b + k] = off;
            off += v[k];
        }
    }
    if (threadIdx.x == kPrefixThreads - 1) {
        const uint64_t S = off;   // the last thread's running sum ends at the grand total
        const uint4 w = philox(0, 0, step, (inst << 8) | kTagResample, key);
        const uint64_t R = ((uint64_t)w.y << 32) | w.x;
        meta[0] = S;
        meta[1] = __umul64hi(R, S);
    }
}

// a(j) = min{a : n * Q_a > j * S + U} for S > 0: binary search over the tile
// ends, then over the tile's local prefix sums.
__device__ __forceinline__ int64_t find_ancestor(int64_t j, int64_t n, int nb, const uint64_t *__restrict__ prefix,
                                                 const uint64_t *__restrict__ total,
                                                 const uint64_t *__restrict__ qloc, uint64_t S, uint64_t U) {
    const unsigned __int128 t = (unsigned __int128)(uint64_t)j * S + U;
    const unsigned __int128 nn = (unsigned __int128)(uint64_t)n;
    // tile: smallest b with n * (prefix[b] + total[b]) > t
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (nn * (prefix[mid] + total[mid]) > t) hi = mid;
        else lo = mid + 1;
    }
    const int b = lo;
    const uint64_t pre = prefix[b];
    int64_t a0 = (int64_t)b * kScanTile;
    int64_t a1 = a0 + kScanTile - 1;
    if (a1 > n - 1) a1 = n - 1;
    while (a0 < a1) {
        const int64_t mid = (a0 + a1) >> 1;
        if (nn * (pre + qloc[mid]) > t) a1 = mid;
        else a0 = mid + 1;
    }
    return a0;
}

// Ancestors of the gather workgroups' range ends: ends[k] = a(k kGatherOut)
// for k < ng and ends[ng] = a(n - 1), one global search per thread (S > 0).
__global__ __launch_bounds__(kRedThreads) void gather_ends_kernel(int64_t n, int nb, int64_t ng,
                                                                  const uint64_t *__restrict__ prefix,
                                                                  const uint64_t *__restrict__ total,
                                                                  const uint64_t *__restrict__ qloc,
                                                                  const uint64_t *__restrict__ meta,
                                                                  int64_t *__restrict__ ends) {
    const int64_t k = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    if (k > ng) return;
    const uint64_t S = meta[0], U = meta[1];
    if (S == 0) return;   // the gather writes its no-ancestor outputs without reading ends
    const int64_t j = k < ng ? k * kGatherOut : n - 1;
    ends[k] = find_ancestor(j, n, nb, prefix, total, qloc, S, U);
}

// Ancestor search fused with the gather of nf 32-bit fields of structure-of-
// arrays state: out[f][j] = in[f][a(j)] (nf = 0: the search alone).  A
// workgroup owns kGatherOut consecutive outputs.  Ancestors are non-decreasing
// in j, so the workgroup's ancestors lie in [ends[k], ends[k + 1]] (the
// ancestors of its first output and of the next workgroup's first output, or
// of the last output): it stages the prefix sums Q_a of that range in LDS with
// coalesced loads and each output binary-searches LDS.  A range longer than
// kGatherStage (a long run of zero weights inside the block) falls back to a
// global search per output; both give the same a(j).  Reads of the state then
// run over consecutive or repeated source words and writes over consecutive
// destination words.  With no ancestor (all weights zero) the outputs are NaN
// words and anc[j] = -1.
__global__ __launch_bounds__(kRedThreads) void ancestor_gather_kernel(
    int64_t n, int nb, const uint64_t *__restrict__ prefix, const uint64_t *__restrict__ total,
    const uint64_t *__restrict__ qloc, const uint64_t *__restrict__ meta, const int64_t *__restrict__ ends, int nf,
    const uint32_t *__restrict__ in, uint32_t *__restrict__ out, int32_t *__restrict__ anc) {
    __shared__ uint64_t sq[kGatherStage];
    const int64_t j0 = (int64_t)blockIdx.x * kGatherOut;
    const uint64_t S = meta[0], U = meta[1];
    if (S == 0) {
        for (int r = 0; r < kGatherPer; ++r) {
            const int64_t j = j0 + r * kRedThreads + threadIdx.x;
            if (j >= n) break;
            if (anc) anc[j] = -1;
            for (int f = 0; f < nf; ++f) out[(size_t)f * n + j] = 0x7fc00000u;
        }
        return;
    }
    const unsigned __int128 nn = (unsigned __int128)(uint64_t)n;
    const int64_t a_lo = ends[blockIdx.x];
    const int64_t range = ends[blockIdx.x + 1] - a_lo + 1;
    const bool staged = range <= kGatherStage;
    if (staged) {
        for (int i = threadIdx.x; i < range; i += kRedThreads) {
            const int64_t a = a_lo + i;
            sq[i] = prefix[a / kScanTile] + qloc[a];
        }
    }
    __syncthreads();
    int64_t a_of[kGatherPer];
#pragma unroll
    for (int r = 0; r < kGatherPer; ++r) {
        const int64_t j = j0 + r * kRedThreads + threadIdx.x;
        a_of[r] = 0;
        if (j >= n) continue;
        if (staged) {
            // smallest i < range with n * Q_{a_lo + i} > j S + U (exists: i = range - 1)
            const unsigned __int128 t = (unsigned __int128)(uint64_t)j * S + U;
            int lo = 0, hi = (int)range - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (nn * sq[mid] > t) hi = mid;
                else lo = mid + 1;
            }
            a_of[r] = a_lo + lo;
        } else {
            a_of[r] = find_ancestor(j, n, nb, prefix, total, qloc, S, U);
        }
        if (anc) anc[j] = (int32_t)a_of[r];
    }
    int f = 0;
    for (; f + 4 <= nf; f += 4) {
        uint32_t v[kGatherPer][4];
#pragma unroll
        for (int r = 0; r < kGatherPer; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                v[r][k] = (j0 + r * kRedThreads + threadIdx.x < n) ? in[(size_t)(f + k) * n + a_of[r]] : 0u;
#pragma unroll
        for (int r = 0; r < kGatherPer; ++r) {
            const int64_t j = j0 + r * kRedThreads + threadIdx.x;
            if (j >= n) continue;
#pragma unroll
            for (int k = 0; k < 4; ++k) out[(size_t)(f + k) * n + j] = v[r][k];
        }
    }
    for (; f < nf; ++f) {
#pragma unroll
        for (int r = 0; r < kGatherPer; ++r) {
            const int64_t j = j0 + r * kRedThreads + threadIdx.x;
            if (j < n) out[(size_t)f * n + j] = in[(size_t)f * n + a_of[r]];
        }
    }
}

// Quantisation, tile scans and the tile prefix with the draw of U: everything
// before the ancestor search.
static int resample_prologue(const void *lw, bool f64, int64_t n, uint64_t seed, uint32_t step, uint32_t inst,
                             const ResampleWs &w, hipStream_t st) {
    const int64_t nb = scan_blocks(n);
    if (int rc = check_grid("quant_scan_kernel", nb, kRedThreads)) return rc;
    const int kb = quant_bits(n);
    const int nm = (int)(nb < kRedBlocksMax ? nb : kRedBlocksMax);
    if (f64) {
        hipLaunchKernelGGL(tile_max_kernel<double>, dim3((unsigned)nm), dim3(kRedThreads), 0, st,
                           (const double *)lw, n, w.blockmax);
        hipLaunchKernelGGL(quant_scan_kernel<double>, dim3((unsigned)nb), dim3(kRedThreads), 0, st,
                           (const double *)lw, n, nm, w.blockmax, kb, w.qloc, w.total);
    } else {
        hipLaunchKernelGGL(tile_max_kernel<float>, dim3((unsigned)nm), dim3(kRedThreads), 0, st,
                           (const float *)lw, n, w.blockmax);
        hipLaunchKernelGGL(quant_scan_kernel<float>, dim3((unsigned)nb), dim3(kRedThreads), 0, st,
                           (const float *)lw, n, nm, w.blockmax, kb, w.qloc, w.total);
    }
    PPL_LAUNCH_CHECK("quant_scan_kernel");
    hipLaunchKernelGGL(tile_prefix_kernel, dim3(1), dim3(kPrefixThreads), 0, st, w.total, (int)nb,
                       make_key(seed), step, inst, w.prefix, w.meta);
    PPL_LAUNCH_CHECK("tile_prefix_kernel");
    return PPL_OK;
}

int run_resample(const void *lw, bool f64, int64_t n, uint64_t seed, uint32_t step, uint32_t inst,
                 int32_t *anc, void *ws, hipStream_t st) {
    return run_resample_gather(lw, f64, n, seed, step, inst, 0, nullptr, nullptr, anc, ws, st);
}

int run_resample_gather(const void *lw, bool f64, int64_t n, uint64_t seed, uint32_t step, uint32_t inst, int nf,
                        const void *state_in, void *state_out, int32_t *anc, void *ws, hipStream_t st) {
    const ResampleWs w = resample_layout(ws, n);
    if (int rc = resample_prologue(lw, f64, n, seed, step, inst, w, st)) return rc;
    const int64_t ng = gather_blocks(n);
    if (int rc = check_grid("ancestor_gather_kernel", ng, kRedThreads)) return rc;
    hipLaunchKernelGGL(gather_ends_kernel, dim3((unsigned)((ng + kRedThreads) / kRedThreads)), dim3(kRedThreads), 0,
                       st, n, (int)scan_blocks(n), ng, w.prefix, w.total, w.qloc, w.meta, w.ends);
    PPL_LAUNCH_CHECK("gather_ends_kernel");
    KernelTimer timer("ancestor_gather_kernel", st);
    hipLaunchKernelGGL(ancestor_gather_kernel, dim3((unsigned)ng), dim3(kRedThreads), 0, st, n,
                       (int)scan_blocks(n), w.prefix, w.total, w.qloc, w.meta, w.ends, nf,
                       (const uint32_t *)state_in, (uint32_t *)state_out, anc);
    timer.stop();
    PPL_LAUNCH_CHECK("ancestor_gather_kernel");
    return PPL_OK;
}

// ------------------------------------------------------------ Philox ----
__global__ __launch_bounds__(256) void philox_fill_kernel(Key key, uint32_t c1, uint32_t c2, uint32_t c3,
                                                          int64_t n, uint4 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = philox((uint32_t)i, c1, c2, c3, key);
}

int run_philox(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t *out, hipStream_t st) {
    const int64_t nb = (n + 255) / 256;
    if (int rc = check_grid("philox_fill_kernel", nb, 256)) return rc;
    hipLaunchKernelGGL(philox_fill_kernel, dim3((unsigned)nb), dim3(256), 0, st, make_key(seed), c1, c2, c3, n,
                       (uint4 *)out);
    PPL_LAUNCH_CHECK("philox_fill_kernel");
    return PPL_OK;
}

}  // namespace ppl
