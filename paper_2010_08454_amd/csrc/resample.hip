// resample.hip -- FP64 log-sum-exp / ESS normaliser, integer-rule systematic
// resampling and the raw Philox stream entry.
//
// The normaliser is the weight normalisation of importance sampling (paper
// Sec. 3.6.2); resampling between factors is the particle-based inference the
// paper names as future work (Sec. 6).  Resampling quantises the weights to
// integers (q_i = floor(exp(lw_i - max) 2^k)) so that the prefix sum, and with
// it every ancestor index, is exact and independent of the reduction order.
#include "device.h"
#include "host.h"
#include "kernels.h"

namespace ppl {

constexpr int kRedThreads = 256;
constexpr int kRedBlocksMax = 1024;
constexpr int kScanItems = 4;                          // items per thread in the scan
constexpr int kScanTile = kRedThreads * kScanItems;    // items per block

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

__global__ __launch_bounds__(64) void lse_finalize_kernel(const double *__restrict__ part, int nb,
                                                          double *__restrict__ out) {
    Partial<0> a = partial_empty<0>();
    for (int b = threadIdx.x; b < nb; b += 64) {
        Partial<0> q = partial_load<0>(part + (size_t)b * 4);
        partial_merge(a, q);
    }
    partial_wave_reduce(a);
    if (threadIdx.x) return;
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
    hipLaunchKernelGGL(lse_finalize_kernel, dim3(1), dim3(64), 0, st, part, (int)nb, out5);
    PPL_LAUNCH_CHECK("lse_finalize_kernel");
    return PPL_OK;
}

// -------------------------------------------------------- resampling ----
// Workspace layout (all 256-byte aligned):
//   blockmax [nb] double | total [nb] u64 | prefix [nb] u64 | meta [4] u64 | qloc [n] u64
struct ResampleWs {
    double *blockmax;
    uint64_t *total, *prefix, *meta, *qloc;
};

static int64_t scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

static ResampleWs resample_layout(void *ws, int64_t n) {
    const int64_t nb = scan_blocks(n);
    char *p = (char *)ws;
    ResampleWs r;
    r.blockmax = (double *)p; p += align_up(nb * sizeof(double), 256);
    r.total = (uint64_t *)p; p += align_up(nb * sizeof(uint64_t), 256);
    r.prefix = (uint64_t *)p; p += align_up(nb * sizeof(uint64_t), 256);
    r.meta = (uint64_t *)p; p += 256;
    r.qloc = (uint64_t *)p;
    return r;
}

size_t resample_ws_bytes(int64_t n) {
    const int64_t nb = scan_blocks(n);
    return align_up(nb * sizeof(double), 256) + 2 * align_up(nb * sizeof(uint64_t), 256) + 256 +
           align_up(n * sizeof(uint64_t), 256);
}

__host__ __device__ inline int quant_bits(int64_t n) {
    int c = 0;
    while (((int64_t)1 << c) < n) ++c;
    return 62 - c;
}

// Exact per-tile maximum (NaN entries are ignored here; run_resample rejects
// NaN through the normaliser's flag).
template <typename T>
__global__ __launch_bounds__(kRedThreads) void tile_max_kernel(const T *__restrict__ lw, int64_t n,
                                                               double *__restrict__ blockmax) {
    __shared__ double red[kRedThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    double m = -INFINITY;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) m = fmax(m, (double)lw[base + k]);
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
// total[b] = tile sum.  Every block first reduces the tile maxima itself.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void quant_scan_kernel(const T *__restrict__ lw, int64_t n, int nb,
                                                                 const double *__restrict__ blockmax, int kbits,
                                                                 uint64_t *__restrict__ qloc,
                                                                 uint64_t *__restrict__ total) {
    __shared__ double smax[kRedThreads / 64];
    __shared__ uint64_t wsum[kRedThreads / 64];
    double m = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) m = fmax(m, blockmax[b]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = m;
    __syncthreads();
    m = smax[0];
#pragma unroll
    for (int w = 1; w < kRedThreads / 64; ++w) m = fmax(m, smax[w]);

    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint64_t q[kScanItems];
    uint64_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t v = 0;
        if (base + k < n) {
            const double e = exp((double)lw[base + k] - m);
            if (e >= 0.0) v = (uint64_t)floor(ldexp(e, kbits));   // NaN entries carry no weight
        }
        run += v;
        q[k] = run;
    }
    const uint64_t incl = wave_inclusive_scan_u64(run);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint64_t off = incl - run;
    for (int w = 0; w < wv; ++w) off += wsum[w];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) qloc[base + k] = q[k] + off;
    if (threadIdx.x == kRedThreads - 1) total[blockIdx.x] = off + run;
}

// Exclusive prefix of the tile totals, S, and U = floor(R S / 2^64).
__global__ __launch_bounds__(kRedThreads) void tile_prefix_kernel(const uint64_t *__restrict__ total, int nb,
                                                                  Key key, uint32_t step, uint32_t inst,
                                                                  uint64_t *__restrict__ prefix,
                                                                  uint64_t *__restrict__ meta) {
    __shared__ uint64_t wsum[kRedThreads / 64];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += kRedThreads) {
        const int b = b0 + threadIdx.x;
        const uint64_t v = b < nb ? total[b] : 0;
        const uint64_t incl = wave_inclusive_scan_u64(v);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        uint64_t off = carry + incl - v;
        for (int w = 0; w < wv; ++w) off += wsum[w];
        if (b < nb) prefix[b] = off;
        __syncthreads();
        if (threadIdx.x == kRedThreads - 1) carry = off + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const uint64_t S = carry;
        const uint4 w = philox(0, 0, step, (inst << 8) | kTagResample, key);
        const uint64_t R = ((uint64_t)w.y << 32) | w.x;
        meta[0] = S;
        meta[1] = __umul64hi(R, S);
    }
}

// a(j) = min{a : n * Q_a > j * S + U}: binary search over the tile ends, then
// over the tile's local prefix sums.
__global__ __launch_bounds__(kRedThreads) void ancestor_search_kernel(
    int64_t n, int nb, const uint64_t *__restrict__ prefix, const uint64_t *__restrict__ total,
    const uint64_t *__restrict__ qloc, const uint64_t *__restrict__ meta, int32_t *__restrict__ anc) {
    const int64_t j = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    if (j >= n) return;
    const uint64_t S = meta[0], U = meta[1];
    if (S == 0) {           // every weight is zero: no ancestor exists
        anc[j] = -1;
        return;
    }
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
    anc[j] = (int32_t)a0;
}

int run_resample(const void *lw, bool f64, int64_t n, uint64_t seed, uint32_t step, uint32_t inst,
                 int32_t *anc, void *ws, hipStream_t st) {
    const int64_t nb = scan_blocks(n);
    if (int rc = check_grid("quant_scan_kernel", nb, kRedThreads)) return rc;
    ResampleWs w = resample_layout(ws, n);
    const int kb = quant_bits(n);
    if (f64) {
        hipLaunchKernelGGL(tile_max_kernel<double>, dim3((unsigned)nb), dim3(kRedThreads), 0, st,
                           (const double *)lw, n, w.blockmax);
        hipLaunchKernelGGL(quant_scan_kernel<double>, dim3((unsigned)nb), dim3(kRedThreads), 0, st,
                           (const double *)lw, n, (int)nb, w.blockmax, kb, w.qloc, w.total);
    } else {
        hipLaunchKernelGGL(tile_max_kernel<float>, dim3((unsigned)nb), dim3(kRedThreads), 0, st,
                           (const float *)lw, n, w.blockmax);
        hipLaunchKernelGGL(quant_scan_kernel<float>, dim3((unsigned)nb), dim3(kRedThreads), 0, st,
                           (const float *)lw, n, (int)nb, w.blockmax, kb, w.qloc, w.total);
    }
    PPL_LAUNCH_CHECK("quant_scan_kernel");
    hipLaunchKernelGGL(tile_prefix_kernel, dim3(1), dim3(kRedThreads), 0, st, w.total, (int)nb,
                       make_key(seed), step, inst, w.prefix, w.meta);
    PPL_LAUNCH_CHECK("tile_prefix_kernel");
    const int64_t sb = (n + kRedThreads - 1) / kRedThreads;
    if (int rc = check_grid("ancestor_search_kernel", sb, kRedThreads)) return rc;
    hipLaunchKernelGGL(ancestor_search_kernel, dim3((unsigned)sb), dim3(kRedThreads), 0, st, n, (int)nb,
                       w.prefix, w.total, w.qloc, w.meta, anc);
    PPL_LAUNCH_CHECK("ancestor_search_kernel");
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
