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
// The nested sites run in two forms.  Pass 1 stays in the log domain: one
// add and one max per path.  Pass 2 runs in the linear domain from one exp
// per prefix: each node carries the weight, relative to M, of the best path
// below it, w = exp(lw_node + V_L[z] - M) <= 1, where V_L[j] is the largest
// log-weight any completion from state j at nested level L can add (a max
// over the suffix, tabulated per state).  A child's weight is the parent's
// times F_L[j][k] = exp(c + V_{L+1}[k] - V_L[j]) <= 1, so no product
// overflows, and a product that underflows belongs to a subtree whose every
// path is below e^-745 of M.  The references set the scale only: every path's
// weight is still formed and added (two FMAs at the last site: into its
// site sum and into the parent's subtotal).
#include "device.h"
#include "host.h"
#include "kernels.h"
#include "timing.h"

namespace ppl {

constexpr int kEnThreads = 128;
constexpr int kEnMaxT = 40;
constexpr int kEnMaxGrid = 2048;
constexpr int kEnMaxC = 1024;            // T K^2 at the path limit (K = 8, T = 16)
constexpr int kEnMaxTS = 12;             // nested sites
constexpr int kEnMaxF = 256;             // TS K^2 factors

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
    double cn[kEnMaxF];          // cn[L][j][k] = c[tail + L][j][k], nested level L (compile-time offsets)
    double F[kEnMaxF];           // F[L][j][k], nested level L (site tail + L)
    double V[(kEnMaxTS + 1) * 8];// V[L][j], V[TS][j] = 0
    double G[kEnMaxTS * 8];      // G[L][j] = sum_k F[L][j][k] (k in order)
    double cm[8];                // cm[j] = max_k cn[TS - 1][j][k] (k in order)
};

// Stages the tables: c for every site, and for the TS nested sites the
// suffix maxima V and the linear-domain factors F (pass 2 only).
template <int K, int TS>
__device__ void en_stage(EnLds &s, const EnumDev &a, bool factors) {
    const int T = a.T, tail = a.tail;
    for (int i = threadIdx.x; i < T * K * K; i += kEnThreads) {
        const int t = i / (K * K), j = (i / K) % K, k = i % K;
        s.c[i] = t == 0 ? 0.0 : a.lA[j * K + k] + a.le[t * K + k];
    }
    if (threadIdx.x < K) s.c0[threadIdx.x] = a.lpi[threadIdx.x] + a.le[threadIdx.x];
    __syncthreads();
    for (int i = threadIdx.x; i < TS * K * K; i += kEnThreads) s.cn[i] = s.c[tail * K * K + i];
    if constexpr (TS > 0)
        if (threadIdx.x < K) {
            const double *row = s.c + ((tail + TS - 1) * K + threadIdx.x) * K;
            double v = row[0];
            for (int k = 1; k < K; ++k) v = fmax(v, row[k]);
            s.cm[threadIdx.x] = v;
        }
    __syncthreads();
    if (!factors) return;
    if (threadIdx.x == 0) {
        for (int j = 0; j < K; ++j) s.V[TS * K + j] = 0.0;
        for (int L = TS - 1; L >= 0; --L)
            for (int j = 0; j < K; ++j) {
                double v = -INFINITY;
                for (int k = 0; k < K; ++k) v = fmax(v, s.c[((tail + L) * K + j) * K + k] + s.V[(L + 1) * K + k]);
                s.V[L * K + j] = v;
            }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TS * K * K; i += kEnThreads) {
        const int L = i / (K * K), j = (i / K) % K, k = i % K;
        const double vj = s.V[L * K + j];
        s.F[i] = vj > -INFINITY ? exp(s.c[((tail + L) * K + j) * K + k] + s.V[(L + 1) * K + k] - vj) : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TS * K; i += kEnThreads) {
        double g = 0.0;
        for (int k = 0; k < K; ++k) g += s.F[i * K + k];
        s.G[i] = g;
    }
    __syncthreads();
}

// Innermost unrolled levels per state count (K^UL paths below the node the
// runtime loops hand over: 64, 81, 64, then K^2).
constexpr int en_ul_max(int K) { return K == 2 ? 6 : K == 3 ? 4 : K == 4 ? 3 : 2; }

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

// ---- pass 1 (log domain).  Levels above TS - UL are runtime loops; the last
// UL levels are unrolled, so their table rows are compile-time indices.
template <int K, int L, int TS, int UL>
struct WalkMax {
    // largest log-weight below a node of an unrolled level
    __device__ static double leafmax(const EnLds &s, int prev, double lw) {
        // Round-to-nearest addition is monotone, so the largest of lw + c_k
        // over the last site's K states is lw plus the largest c_k: the same
        // double as taking the K sums and their maximum.
        if constexpr (L == TS - 1) {
            return lw + s.cm[prev];
        } else {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double x = WalkMax<K, L + 1, TS, UL>::leafmax(s, k, lw + s.cn[(L * K + prev) * K + k]);
                v = k == 0 ? x : fmax(v, x);
            }
            return v;
        }
    }
    // Raises best to the largest log-weight below the node and, when it does,
    // records the index of the node at level TS - UL that holds it.
    __device__ static void run(const EnLds &s, int prev, double lw, uint64_t idx, double &best, uint64_t &bnode) {
        if constexpr (L < TS - UL) {
#pragma unroll 1
            for (int k = 0; k < K; ++k)
                WalkMax<K, L + 1, TS, UL>::run(s, k, lw + s.cn[(L * K + prev) * K + k], idx * K + k, best, bnode);
        } else {
            const double v = leafmax(s, prev, lw);
            if (v > best) {
                best = v;
                bnode = idx;
            }
        }
    }
};

// The path index of the largest log-weight v below node `node` (at level
// TS - UL) of prefix p: the node's log-weight is re-summed in the walk's
// order, then the first of its K^UL completions that reaches v is found.
template <int K, int TS, int UL>
__device__ uint64_t en_locate(const EnLds &s, int tail, uint64_t p, uint64_t node, double v) {
    constexpr int NL = TS - UL;                  // runtime levels above the node
    constexpr int n = (int)ipow(K, UL);
    int prev;
    double lw = en_prefix<K>(s, tail, p, prev);
    uint64_t div = ipow(K, NL) / K;
    for (int L = 0; L < NL; ++L, div /= K) {
        const int k = (int)((node / div) % K);
        lw = lw + s.cn[(L * K + prev) * K + k];
        prev = k;
    }
    int m = 0;
    for (; m < n - 1; ++m) {
        double x = lw;
        int pv = prev, r = m;
        for (int d = 0, dv = n / K; d < UL; ++d, dv /= K) {
            const int k = r / dv;
            r -= k * dv;
            x = x + s.cn[((NL + d) * K + pv) * K + k];
            pv = k;
        }
        if (x == v) break;
    }
    return (p * ipow(K, NL) + node) * n + m;
}

// ---- pass 2 (linear domain): returns the sum of the path weights below the
// node and adds each nested site's share to marg.
template <int K, int L, int TS, int UL>
struct WalkSum {
    __device__ static double run(const EnLds &s, int prev, double w, double (&marg)[TS][K]) {
        const double *F = s.F + (L * K + prev) * K;
        double tot = 0.0;
        if constexpr (L < TS - UL) {
#pragma unroll 1
            for (int k = 0; k < K; ++k) {
                const double sub = WalkSum<K, L + 1, TS, UL>::run(s, k, w * F[k], marg);
#pragma unroll
                for (int kk = 0; kk < K; ++kk) marg[L][kk] += (k == kk) ? sub : 0.0;
                tot += sub;
            }
        } else if constexpr (L == TS - 1) {
            // each path's weight w F[k] goes into its site sum; the node's
            // subtotal, their sum, is w times the row sum G (one product for
            // the K paths)
#pragma unroll
            for (int k = 0; k < K; ++k) marg[L][k] = fma(w, F[k], marg[L][k]);
            tot = w * s.G[L * K + prev];
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double sub = WalkSum<K, L + 1, TS, UL>::run(s, k, w * F[k], marg);
                marg[L][k] += sub;
                tot += sub;
            }
        }
        return tot;
    }
};

// Pass 1: the largest log-weight and its path.
template <int K, int TS, int UL>
__global__ __launch_bounds__(kEnThreads) void enum_max_kernel(EnumDev a) {
    __shared__ EnLds s;
    __shared__ double s_best[kEnThreads];
    __shared__ uint64_t s_idx[kEnThreads];
    en_stage<K, TS>(s, a, false);
    double best = -INFINITY;
    uint64_t bidx = 0, bp = 0, bnode = 0;
    for (uint64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const uint64_t p = tile * kEnThreads + threadIdx.x;
        if (p >= a.n_prefix) continue;
        int last;
        const double lw = en_prefix<K>(s, a.tail, p, last);
        if constexpr (TS == 0) {
            if (lw > best) { best = lw; bidx = p; }
        } else {
            const double before = best;
            uint64_t node = 0;
            WalkMax<K, 0, TS, UL>::run(s, last, lw, 0, best, node);
            if (best > before) {
                bp = p;
                bnode = node;
            }
        }
    }
    if constexpr (TS > 0)
        if (best > -INFINITY) bidx = en_locate<K, TS, UL>(s, a.tail, bp, bnode, best);
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
template <int K, int TS, int UL>
__global__ __launch_bounds__(kEnThreads) void enum_sum_kernel(EnumDev a) {
    constexpr int TSA = TS > 0 ? TS : 1;
    constexpr int kWaves = kEnThreads / 64;
    __shared__ EnLds s;
    __shared__ double s_sub[kEnThreads];
    __shared__ double s_wsum[kWaves];
    en_stage<K, TS>(s, a, true);
    const double M = a.glob[0];
    const bool skip = !(M > -INFINITY) || a.glob[2] != 0.0;
    const int tail = a.tail, T = a.T;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
                const double w = exp(lw + s.V[last] - M);      // the best path below the prefix, <= 1
                sub = WalkSum<K, 0, TS, UL>::run(s, last, w, marg);
            }
        }
        tot += sub;
        // the tile's total, the same bits in every lane (butterfly of commutative adds)
        double ws = sub;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) ws += __shfl_xor(ws, o);
        s_sub[threadIdx.x] = sub;
        if (lane == 0) s_wsum[wave] = ws;
        __syncthreads();
        double tile_tot = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) tile_tot += s_wsum[w];
        // prefix site t of prefix base + i has digit (q + (r + i) div pw) mod K, q and r from base = q pw + r
#pragma unroll
        for (int j = 0; j < kOwn; ++j) {
            const int e = threadIdx.x + j * kEnThreads;
            if (e < tail * K) {
                const int t = e / K, k = e - t * K;
                uint64_t pw = 1;
                for (int u = t + 1; u < tail; ++u) pw *= K;
                const uint64_t q = base / pw, r = base - q * pw;
                const int qm = (int)(q % K);
                double acc = 0.0;
                if (pw - r >= (uint64_t)kEnThreads) {
                    acc = qm == k ? tile_tot : 0.0;          // one digit over the whole tile
                } else if (pw >= (uint64_t)kEnThreads) {
                    // the digit steps once, at c = pw - r
                    const int c = (int)(pw - r);
                    if (qm == k)
                        for (int i = 0; i < c; ++i) acc += s_sub[i];
                    if ((qm + 1) % K == k)
                        for (int i = c; i < kEnThreads; ++i) acc += s_sub[i];
                } else {
                    // runs of pw prefixes per digit: those of digit k start at n pw - r, n = (k - qm) mod K + K i
                    const int pw32 = (int)pw, r32 = (int)r;
                    for (int n = (k - qm + K) % K; n * pw32 - r32 < kEnThreads; n += K) {
                        const int lo = max(0, n * pw32 - r32), hi = min(kEnThreads, (n + 1) * pw32 - r32);
                        for (int i = lo; i < hi; ++i) acc += s_sub[i];
                    }
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
// 5^5, 6^5, 7^4, 8^4).
constexpr int en_ts_max(int K) { return K == 2 ? 12 : K == 3 ? 7 : K == 4 ? 6 : K <= 6 ? 5 : 4; }
constexpr int en_ul(int K, int ts) { return std::min(en_ul_max(K), ts); }

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
    constexpr int UL = en_ul(K, TS);
    static_assert(TS <= kEnMaxTS && TS * K * K <= kEnMaxF, "nested tables exceed their LDS slots");
    {
        KernelTimer timer("enum_max_kernel", st);
        hipLaunchKernelGGL((enum_max_kernel<K, TS, UL>), dim3((unsigned)p.grid), dim3(kEnThreads), 0, st, d);
        timer.stop();
    }
    PPL_LAUNCH_CHECK("enum_max_kernel");
    hipLaunchKernelGGL(enum_merge_kernel, dim3(1), dim3(256), 0, st, d.rec1, p.grid, d.le, d.T * K, d.glob);
    PPL_LAUNCH_CHECK("enum_merge_kernel");
    {
        KernelTimer timer("enum_sum_kernel", st);
        hipLaunchKernelGGL((enum_sum_kernel<K, TS, UL>), dim3((unsigned)p.grid), dim3(kEnThreads), 0, st, d);
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
