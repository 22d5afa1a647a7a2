// enumerate.hip -- exact inference by enumeration (paper Sec. 3.6.1) on the
// GPU: every execution of a model whose sample sites all have finite support,
// weighted by its sample probabilities and factors.
//
// Model: a hidden Markov chain of K states over T steps, z_0 ~ Cat(pi0),
// z_t ~ Cat(A[z_{t-1}]), observe(Normal(mu[z_t], sigma), y_t).  An execution
// is a path; the paths form the support product {0..K-1}^T, indexed by
// sum_t z_t K^(T-1-t).  A path's log-weight is the sum over sites of
// c_t(z_{t-1}, z_t) = log A[z_{t-1}][z_t] + log N(y_t; mu[z_t], sigma) (site 0:
// log pi0[z_0] + its emission).
//
// The paper enumerates breadth first, resuming an execution at a sample site
// once for every value of its support.  Here the first T - Ts sites (the
// prefix) are fanned out over threads, a prefix per thread and 128 prefixes
// per tile, workgroups striding over the tiles; a thread resumes its prefix
// for every value of the last Ts sites in nested loops fixed at compile time.
// Two passes over the paths: the first finds the largest log-weight M and the
// most probable path (the lowest index among equals), the second sums
// exp(lw - M) in total and per (t, z_t): the nested sites' sums in
// registers, the prefix sites' per tile through LDS into one owner thread per
// (t, k).  Records are merged in workgroup order, so results do not depend on
// timing.
//
// The last BD sites form a block whose K^BD suffixes are tabulated per state
// j before it: their log-weights b[j][m] (the sum of c over the block's sites)
// and, for the second pass, f[j][m] = exp(b[j][m] - q[j]) with q[j] = max_m
// b[j][m].  Pass 1 then costs one add and one max per path; pass 2 takes one
// exp per block, G = exp(lw_j + q[j] - M) (the weight of the block's best
// path, at most 1, so it cannot overflow), and two fused multiply-adds per
// path (G f[j][m] into its last site's sum and into the block subtotal).
#include "device.h"
#include "host.h"
#include "kernels.h"
#include "timing.h"

namespace ppl {

constexpr int kEnThreads = 128;
constexpr int kEnMaxT = 40;
constexpr int kEnMaxGrid = 2048;
constexpr int kEnMaxC = 1024;            // T K^2 at the path limit (K = 8, T = 16)
constexpr int kEnMaxB = 512;             // K^(BD + 1)

__host__ __device__ constexpr uint64_t ipow(uint64_t b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

struct EnumDev {
    int T, tail;                 // sites, prefix sites (T - Ts)
    uint64_t n_prefix;           // K^tail
    uint64_t n_tiles;            // ceil(n_prefix / kEnThreads)
    const double *le;            // [T][K] log emission densities
    double lpi[8], lA[64];
    double *rec1;                // [grid][2] pass-1 records {best lw, best index (bits)}
    double *glob;                // [3] {M, best index (bits), non-finite}
    double *rec2;                // [grid][1 + T K] pass-2 records {total, per-site sums}
};

struct EnLds {
    double c[kEnMaxC];           // c[t][j][k], t >= 1
    double c0[8];                // site 0: log pi0[k] + le[0][k]
    double b[kEnMaxB];           // block log-weights b[j][m]
    double f[kEnMaxB];           // block factors f[j][m]
    double q[8];
};

template <int K, int BD>
__device__ void en_stage(EnLds &s, const EnumDev &a) {
    constexpr int KB = (int)ipow(K, BD);
    const int T = a.T;
    for (int i = threadIdx.x; i < T * K * K; i += kEnThreads) {
        const int t = i / (K * K), j = (i / K) % K, k = i % K;
        s.c[i] = t == 0 ? 0.0 : a.lA[j * K + k] + a.le[t * K + k];
    }
    if (threadIdx.x < K) s.c0[threadIdx.x] = a.lpi[threadIdx.x] + a.le[threadIdx.x];
    __syncthreads();
    {
        // suffix m of the block (digits over sites T - BD .. T - 1) after state j
        for (int i = threadIdx.x; i < K * KB; i += kEnThreads) {
            const int j = i / KB;
            int m = i % KB, prev = j, div = KB / K;      // BD = 0: the empty suffix, b = 0, f = 1
            double v = 0.0;
            for (int d = 0; d < BD; ++d) {
                const int k = m / div;
                m -= k * div;
                div /= K;
                v += s.c[(T - BD + d) * K * K + prev * K + k];
                prev = k;
            }
            s.b[i] = v;
        }
        __syncthreads();
        if (threadIdx.x < K) {
            double q = -INFINITY;
            for (int m = 0; m < KB; ++m) q = fmax(q, s.b[threadIdx.x * KB + m]);
            s.q[threadIdx.x] = q;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < K * KB; i += kEnThreads) {
            const double q = s.q[i / KB];
            s.f[i] = q > -INFINITY ? exp(s.b[i] - q) : 0.0;
        }
    }
    __syncthreads();
}

// ---- pass 1: nested loops over the last TS sites.  Levels above the block's
// root are runtime loops; the root level (TS - BD - 1) is unrolled so the
// block's table row j is a compile-time index.
template <int K, int BD, int D>
struct BlockMax {
    // largest log-weight of the block under state j with log-weight lw
    __device__ static double run(const double *b, int m0, double lw) {
        double v = -INFINITY;
#pragma unroll
        for (int k = 0; k < K; ++k) v = fmax(v, BlockMax<K, BD, D + 1>::run(b, m0 * K + k, lw));
        return v;
    }
};
template <int K, int BD>
struct BlockMax<K, BD, BD> {
    __device__ static double run(const double *b, int m, double lw) { return lw + b[m]; }
};

template <int K, int L, int TS, int BD>
struct WalkMax {
    __device__ static void run(const EnLds &s, int t, int prev, double lw, uint64_t idx, double &best,
                               uint64_t &bidx) {
        constexpr int KB = (int)ipow(K, BD);
        if constexpr (L < TS - BD - 1) {
#pragma unroll 1
            for (int k = 0; k < K; ++k)
                WalkMax<K, L + 1, TS, BD>::run(s, t + 1, k, lw + s.c[(t * K + prev) * K + k], idx * K + k, best,
                                               bidx);
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double lwj = lw + s.c[(t * K + prev) * K + j];
                const double v = BlockMax<K, BD, 0>::run(s.b + j * KB, 0, lwj);
                if (v > best) {
                    int m = 0;
                    while (m < KB - 1 && lwj + s.b[j * KB + m] != v) ++m;   // the first suffix reaching it
                    best = v;
                    bidx = (idx * K + j) * KB + m;
                }
            }
        }
    }
};

// ---- pass 2: the same loops; the block's paths in the linear domain.
template <int K, int TS, int BD, int D>
struct BlockSum {
    // sum of the block's path weights G f[m] under suffix prefix m0, adding each site's share to marg
    __device__ static double run(const double *f, int m0, double G, double (&marg)[TS][K]) {
        double tot = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if constexpr (D == BD - 1) {
                const double w = f[m0 * K + k];
                marg[TS - 1][k] = fma(G, w, marg[TS - 1][k]);
                tot = fma(G, w, tot);
            } else {
                const double sub = BlockSum<K, TS, BD, D + 1>::run(f, m0 * K + k, G, marg);
                marg[TS - BD + D][k] += sub;
                tot += sub;
            }
        }
        return tot;
    }
};

template <int K, int L, int TS, int BD>
struct WalkSum {
    __device__ static double run(const EnLds &s, int t, int prev, double lw, double M, double (&marg)[TS][K]) {
        constexpr int KB = (int)ipow(K, BD);
        double tot = 0.0;
        if constexpr (L < TS - BD - 1) {
#pragma unroll 1
            for (int k = 0; k < K; ++k) {
                const double sub =
                    WalkSum<K, L + 1, TS, BD>::run(s, t + 1, k, lw + s.c[(t * K + prev) * K + k], M, marg);
#pragma unroll
                for (int kk = 0; kk < K; ++kk) marg[L][kk] += (k == kk) ? sub : 0.0;
                tot += sub;
            }
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double G = exp(lw + s.c[(t * K + prev) * K + j] + s.q[j] - M);
                double sub = G;
                if constexpr (BD > 0) sub = BlockSum<K, TS, BD, 0>::run(s.f + j * KB, 0, G, marg);
                marg[L][j] += sub;
                tot += sub;
            }
        }
        return tot;
    }
};

// Log-weight of prefix p (its digits are sites 0..tail-1) and its last state.
template <int K>
__device__ __forceinline__ double en_prefix(const EnLds &s, int tail, uint64_t p, int &last) {
    int z[kEnMaxT];
    for (int t = tail - 1; t >= 0; --t) {
        z[t] = (int)(p % K);
        p /= K;
    }
    double lw = s.c0[z[0]];
    for (int t = 1; t < tail; ++t) lw += s.c[(t * K + z[t - 1]) * K + z[t]];
    last = z[tail - 1];
    return lw;
}

// Pass 1: the largest log-weight and its path.
template <int K, int TS, int BD>
__global__ __launch_bounds__(kEnThreads) void enum_max_kernel(EnumDev a) {
    __shared__ EnLds s;
    __shared__ double s_best[kEnThreads];
    __shared__ uint64_t s_idx[kEnThreads];
    en_stage<K, BD>(s, a);
    constexpr uint64_t kts = ipow(K, TS);
    double best = -INFINITY;
    uint64_t bidx = 0;
    for (uint64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const uint64_t p = tile * kEnThreads + threadIdx.x;
        if (p >= a.n_prefix) continue;
        int last;
        const double lw = en_prefix<K>(s, a.tail, p, last);
        if constexpr (TS == 0) {
            if (lw > best) { best = lw; bidx = p; }
        } else {
            double bl = -INFINITY;
            uint64_t bi = 0;
            WalkMax<K, 0, TS, BD>::run(s, a.tail, last, lw, 0, bl, bi);
            if (bl > best) { best = bl; bidx = p * kts + bi; }
        }
    }
    s_best[threadIdx.x] = best;
    s_idx[threadIdx.x] = bidx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double bl = -INFINITY;
        uint64_t bi = 0;
        for (int i = 0; i < kEnThreads; ++i)
            if (s_best[i] > bl || (s_best[i] == bl && s_idx[i] < bi)) { bl = s_best[i]; bi = s_idx[i]; }
        double *r = a.rec1 + 2 * (size_t)blockIdx.x;
        r[0] = bl;
        r[1] = __longlong_as_double((long long)bi);
    }
}

// Merges the pass-1 records (the largest log-weight, the lowest index among
// equals) and flags a NaN emission term (a NaN observation makes every path's
// log-weight NaN).  One workgroup.
__global__ __launch_bounds__(256) void enum_merge_kernel(const double *__restrict__ rec1, int nrec,
                                                         const double *__restrict__ le, int n_le,
                                                         double *__restrict__ glob) {
    __shared__ double s_best[256];
    __shared__ uint64_t s_idx[256];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    double bl = -INFINITY;
    uint64_t bi = 0;
    for (int r = threadIdx.x; r < nrec; r += 256) {
        const double b = rec1[2 * (size_t)r];
        const uint64_t i = (uint64_t)__double_as_longlong(rec1[2 * (size_t)r + 1]);
        if (b > bl || (b == bl && i < bi)) { bl = b; bi = i; }
    }
    int bad = 0;
    for (int i = threadIdx.x; i < n_le; i += 256) bad |= le[i] != le[i];
    if (bad) atomicOr(&s_bad, 1);
    s_best[threadIdx.x] = bl;
    s_idx[threadIdx.x] = bi;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256; ++i)
            if (s_best[i] > bl || (s_best[i] == bl && s_idx[i] < bi)) { bl = s_best[i]; bi = s_idx[i]; }
        glob[0] = bl;
        glob[1] = __longlong_as_double((long long)bi);
        glob[2] = s_bad ? 1.0 : 0.0;
    }
}

// Pass 2: sums of exp(lw - M) in total and per (t, z_t).
template <int K, int TS, int BD>
__global__ __launch_bounds__(kEnThreads) void enum_sum_kernel(EnumDev a) {
    constexpr int TSA = TS > 0 ? TS : 1;
    __shared__ EnLds s;
    __shared__ double s_sub[kEnThreads];
    en_stage<K, BD>(s, a);
    const double M = a.glob[0];
    const bool skip = !(M > -INFINITY) || a.glob[2] != 0.0;
    const int tail = a.tail, T = a.T;
    double *rec = a.rec2 + (size_t)blockIdx.x * (1 + T * K);
    // owner entries e = t K + k of the prefix sites: this thread owns e = threadIdx.x + j kEnThreads
    constexpr int kOwn = (kEnMaxT * 8 + kEnThreads - 1) / kEnThreads;
    double own[kOwn];
#pragma unroll
    for (int j = 0; j < kOwn; ++j) own[j] = 0.0;
    double marg[TSA][K];
#pragma unroll
    for (int l = 0; l < TSA; ++l)
#pragma unroll
        for (int k = 0; k < K; ++k) marg[l][k] = 0.0;
    double tot = 0.0;
    for (uint64_t tile = blockIdx.x; !skip && tile < a.n_tiles; tile += gridDim.x) {
        const uint64_t base = tile * kEnThreads;
        const uint64_t p = base + threadIdx.x;
        double sub = 0.0;
        if (p < a.n_prefix) {
            int last;
            const double lw = en_prefix<K>(s, tail, p, last);
            if constexpr (TS == 0) {
                sub = exp(lw - M);
            } else {
                sub = WalkSum<K, 0, TS, BD>::run(s, tail, last, lw, M, marg);
            }
        }
        tot += sub;
        s_sub[threadIdx.x] = sub;
        __syncthreads();
        // prefix site t has digit q (mod K) for threads i < c and q + 1 after (c = K^(tail-1-t) - base mod it)
#pragma unroll
        for (int j = 0; j < kOwn; ++j) {
            const int e = threadIdx.x + j * kEnThreads;
            if (e < tail * K) {
                const int t = e / K, k = e - t * K;
                uint64_t pw = 1;
                for (int u = t + 1; u < tail; ++u) pw *= K;
                const uint64_t q = base / pw, r = base - q * pw;
                double acc = 0.0;
                if (pw >= kEnThreads) {
                    const int c = (int)std::min<uint64_t>(pw - r, kEnThreads);
                    const int d0 = (int)(q % K), d1 = (int)((q + 1) % K);
                    if (d0 == k)
                        for (int i = 0; i < c; ++i) acc += s_sub[i];
                    if (d1 == k)
                        for (int i = c; i < kEnThreads; ++i) acc += s_sub[i];
                } else {
                    const uint32_t pw32 = (uint32_t)pw, r32 = (uint32_t)r, qm = (uint32_t)(q % K);
                    for (int i = 0; i < kEnThreads; ++i)
                        if ((qm + (r32 + (uint32_t)i) / pw32) % K == (uint32_t)k) acc += s_sub[i];
                }
                own[j] += acc;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kOwn; ++j) {
        const int e = threadIdx.x + j * kEnThreads;
        if (e < tail * K) rec[1 + e] = own[j];
    }
    // the total and the nested sites, one value at a time through LDS, thread order
    s_sub[threadIdx.x] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int i = 0; i < kEnThreads; ++i) acc += s_sub[i];
        rec[0] = acc;
    }
#pragma unroll
    for (int l = 0; l < TS; ++l) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            __syncthreads();
            s_sub[threadIdx.x] = marg[l][k];
            __syncthreads();
            if (threadIdx.x == 0) {
                double acc = 0.0;
                for (int i = 0; i < kEnThreads; ++i) acc += s_sub[i];
                rec[1 + (tail + l) * K + k] = acc;
            }
        }
    }
}

// Merges the pass-2 records in record order: scal[4] = {log Z, paths, log
// joint of the most probable path, status}, marg[T][K] = P(z_t = k | y),
// map[T] the most probable path.
__global__ __launch_bounds__(256) void enum_finalize_kernel(const double *__restrict__ rec2, int nrec, int K, int T,
                                                            double paths, const double *__restrict__ glob,
                                                            double *__restrict__ scal, double *__restrict__ marg,
                                                            int32_t *__restrict__ map) {
    __shared__ double s_tot;
    const int rl = 1 + T * K;
    const double M = glob[0];
    const int status = glob[2] != 0.0 ? PPL_E_NONFINITE : M > -INFINITY ? PPL_OK : PPL_E_ZERO_WEIGHT;
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int r = 0; r < nrec; ++r) acc += rec2[(size_t)r * rl];
        s_tot = acc;
    }
    __syncthreads();
    const double tot = s_tot;
    if (marg)
        for (int f = threadIdx.x; f < T * K; f += blockDim.x) {
            double acc = 0.0;
            for (int r = 0; r < nrec; ++r) acc += rec2[(size_t)r * rl + 1 + f];
            marg[f] = status == PPL_OK ? acc / tot : 0.0;
        }
    if (threadIdx.x == 0) {
        scal[0] = status == PPL_OK ? M + log(tot) : status == PPL_E_NONFINITE ? NAN : -INFINITY;
        scal[1] = paths;
        scal[2] = status == PPL_OK ? M : scal[0];
        scal[3] = (double)status;
        if (map) {
            uint64_t q = (uint64_t)__double_as_longlong(glob[1]);
            for (int t = T - 1; t >= 0; --t) { map[t] = (int32_t)(q % (uint64_t)K); q /= (uint64_t)K; }
        }
    }
}

struct EnEmission {
    double mu[8];
    double sigma;
};

// log emission densities le[t][k] = log Normal(y_t; mu_k, sigma).
__global__ void enum_emission_kernel(const double *__restrict__ y, int T, int K, EnEmission e,
                                     double *__restrict__ le) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T * K) return;
    const int t = i / K, k = i % K;
    const double r = (y[t] - e.mu[k]) / e.sigma;
    le[i] = -0.5 * log(2.0 * M_PI) - log(e.sigma) - 0.5 * r * r;
}

// ---------------------------------------------------------------- host --
// Nested sites per state count (the paths below a prefix: 2^12, 3^7, 4^6,
// 5^5, 6^5, 7^4, 8^4) and block sites (suffixes per state: 16, 27, then K^2).
constexpr int en_ts_max(int K) { return K == 2 ? 12 : K == 3 ? 7 : K == 4 ? 6 : K <= 6 ? 5 : 4; }
constexpr int en_bd_max(int K) { return K == 2 ? 4 : K == 3 ? 3 : 2; }
constexpr int en_bd(int K, int ts) { return ts <= 1 ? 0 : std::min(en_bd_max(K), ts - 1); }

struct EnPlan {
    int Ts, tail, grid;
    uint64_t n_prefix, n_tiles;
};

static int en_plan(int K, int T, EnPlan &p) {
    if (K < 1 || K > 8 || T < 1 || T > kEnMaxT || T * K * K > kEnMaxC)
        return fail(PPL_E_UNSUPPORTED, "no enumeration plan for %d states over %d steps", K, T);
    p.Ts = K == 1 ? 0 : std::min(en_ts_max(K), T - 1);   // site 0 is always a prefix site
    p.tail = T - p.Ts;
    p.n_prefix = ipow((uint64_t)K, p.tail);
    p.n_tiles = (p.n_prefix + kEnThreads - 1) / kEnThreads;
    p.grid = (int)std::min<uint64_t>(p.n_tiles, kEnMaxGrid);
    return PPL_OK;
}

// Workspace: [256 scalars][le T K][glob 3][rec1 grid 2][rec2 grid (1 + T K)], each 256-byte aligned.
size_t enum_ws_bytes(int K, int T) {
    EnPlan p;
    if (en_plan(K, T, p)) return 0;
    return 256 + align_up((size_t)T * K * 8, 256) + 256 + align_up((size_t)p.grid * 2 * 8, 256) +
           align_up((size_t)p.grid * (1 + T * K) * 8, 256);
}

template <int K, int TS>
static int en_launch(const EnumDev &d, const EnPlan &p, hipStream_t st) {
    constexpr int BD = en_bd(K, TS);
    static_assert(ipow(K, BD + 1) <= kEnMaxB, "block table exceeds its LDS slot");
    {
        KernelTimer timer("enum_max_kernel", st);
        hipLaunchKernelGGL((enum_max_kernel<K, TS, BD>), dim3((unsigned)p.grid), dim3(kEnThreads), 0, st, d);
        timer.stop();
    }
    PPL_LAUNCH_CHECK("enum_max_kernel");
    hipLaunchKernelGGL(enum_merge_kernel, dim3(1), dim3(256), 0, st, d.rec1, p.grid, d.le, d.T * K, d.glob);
    PPL_LAUNCH_CHECK("enum_merge_kernel");
    {
        KernelTimer timer("enum_sum_kernel", st);
        hipLaunchKernelGGL((enum_sum_kernel<K, TS, BD>), dim3((unsigned)p.grid), dim3(kEnThreads), 0, st, d);
        timer.stop();
    }
    PPL_LAUNCH_CHECK("enum_sum_kernel");
    return PPL_OK;
}

template <int K, int TS = en_ts_max(K)>
static int en_dispatch(const EnumDev &d, const EnPlan &p, hipStream_t st) {
    if (p.Ts == TS) return en_launch<K, TS>(d, p, st);
    if constexpr (TS > 0) return en_dispatch<K, TS - 1>(d, p, st);
    return fail(PPL_E_UNSUPPORTED, "no enumeration kernel for %d states with %d nested sites", K, p.Ts);
}

int run_enumerate_hmm(const EnumArgs &a, hipStream_t st) {
    const int K = a.K, T = a.T;
    EnPlan p;
    if (int rc = en_plan(K, T, p)) return rc;
    char *w = (char *)a.ws + 256;             // the first 256 bytes hold the scalars when the caller passes none
    double *le = (double *)w;
    w += align_up((size_t)T * K * 8, 256);
    double *glob = (double *)w;
    w += 256;
    double *rec1 = (double *)w;
    w += align_up((size_t)p.grid * 2 * 8, 256);
    double *rec2 = (double *)w;
    EnEmission em{};
    for (int k = 0; k < K; ++k) em.mu[k] = a.mu[k];
    em.sigma = a.sigma;
    hipLaunchKernelGGL(enum_emission_kernel, dim3((T * K + 255) / 256), dim3(256), 0, st, a.y, T, K, em, le);
    PPL_LAUNCH_CHECK("enum_emission_kernel");
    EnumDev d{};
    d.T = T;
    d.tail = p.tail;
    d.n_prefix = p.n_prefix;
    d.n_tiles = p.n_tiles;
    d.le = le;
    d.rec1 = rec1;
    d.glob = glob;
    d.rec2 = rec2;
    for (int k = 0; k < K; ++k) d.lpi[k] = log(a.pi0[k]);
    for (int k = 0; k < K * K; ++k) d.lA[k] = log(a.A[k]);
    int rc = PPL_E_ARG;
    switch (K) {
        case 1: rc = en_launch<1, 0>(d, p, st); break;
        case 2: rc = en_dispatch<2>(d, p, st); break;
        case 3: rc = en_dispatch<3>(d, p, st); break;
        case 4: rc = en_dispatch<4>(d, p, st); break;
        case 5: rc = en_dispatch<5>(d, p, st); break;
        case 6: rc = en_dispatch<6>(d, p, st); break;
        case 7: rc = en_dispatch<7>(d, p, st); break;
        case 8: rc = en_dispatch<8>(d, p, st); break;
    }
    if (rc) return rc;
    hipLaunchKernelGGL(enum_finalize_kernel, dim3(1), dim3(256), 0, st, rec2, p.grid, K, T,
                       (double)ipow((uint64_t)K, T), glob, a.scalars, a.marginals, a.map);
    PPL_LAUNCH_CHECK("enum_finalize_kernel");
    return PPL_OK;
}

}  // namespace ppl
