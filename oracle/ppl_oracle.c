/*
 * ppl_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may load, link or
 * call this library: only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * constant with the HIP library; the only contract the two sides share is the
 * written random-stream specification (Philox4x32-10 counter layout, uniform
 * and Box-Muller conversions), which each side implements on its own.
 *
 * What it computes, and where the paper defines it:
 *   - sample / factor / observe semantics: a particle draws its latents at the
 *     model's sample sites and adds log-factors to its log-weight
 *     (paper Sec. 3.4, figure "sample-factor-observe-impl").
 *   - importance sampling: run the model N times, each run's sample/factor
 *     calls give it a log-probability, normalise those over the runs
 *     (paper Sec. 3.6.2).
 *   - the polynomial model of the paper's running example (Sec. 1.1, figure
 *     "ppl-example2"): degree from a uniform-discrete prior, Gaussian
 *     coefficients, factor(-distance).
 *   - particle-based inference (SMC), named as future work in Sec. 6: bootstrap
 *     propagation, log-sum-exp normaliser, ESS trigger, systematic resampling.
 *   - fixed-size distribution/state values (Sec. 4.2.2, 4.2.4): every model here
 *     has a static maximum latent size.
 * All arithmetic is IEEE double, built with -ffp-contract=off, in the order the
 * definitions state.  Particle loops are independent and may run on several
 * host threads (OpenMP); every reduction runs sequentially in particle order
 * with Neumaier-compensated sums.
 *
 * Philox4x32-10 follows Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers:
 * As Easy as 1, 2, 3" (SC'11): ten rounds of the Philox S-box on a 4x32-bit
 * counter with a 2x32-bit key bumped by the golden-ratio / sqrt(3)-1 Weyl
 * constants between rounds.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- Philox -- */
/* Round multipliers and Weyl key increments of Philox4x32 (SC'11, Table 2 / Sec. 4). */
#define PHX_MUL_A 0xD2511F53u
#define PHX_MUL_B 0xCD9E8D57u
#define PHX_WEYL_A 0x9E3779B9u
#define PHX_WEYL_B 0xBB67AE85u

/* One Philox4x32-10 block: counter (c0,c1,c2,c3), key = (lo32(seed), hi32(seed)). */
void or_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
               uint64_t seed, uint32_t out[4])
{
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHX_WEYL_A; k1 += PHX_WEYL_B; }
        uint64_t pa = (uint64_t)PHX_MUL_A * x0;
        uint64_t pb = (uint64_t)PHX_MUL_B * x2;
        uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)pb;
        uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)pa;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Batch form for tests: ctr is [n][4], seeds is [n] (one key per row). */
void or_philox_batch(int64_t n, const uint32_t *ctr, const uint64_t *seeds, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        or_philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], seeds[i], out + 4 * i);
}

/* Stream tags carried in the low byte of counter word 3 (instance id above it). */
enum { TAG_PRIOR = 0, TAG_PROPOSAL = 1, TAG_RESAMPLE = 2, TAG_TRAIN_SIM = 4,
       TAG_INIT_WEIGHTS = 5 };

static inline void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                         uint32_t inst, uint32_t tag, uint32_t w[4])
{
    or_philox(c0, c1, c2, (inst << 8) | tag, seed, w);
}

/* ------------------------------------------------------------- uniforms -- */
/* Single-precision stream uniform: 23 high bits plus one half, exact in FP32. */
double or_u01_single(uint32_t w) { return ((double)(w >> 9) + 0.5) * 0x1p-23; }

/* Double-precision stream uniform from two words (lo first): 52 bits plus a half. */
double or_u01_double(uint32_t lo, uint32_t hi)
{
    uint64_t v = ((uint64_t)hi << 32) | lo;
    return ((double)(v >> 12) + 0.5) * 0x1p-52;
}

/* Box-Muller: radius sqrt(-2 ln u1), angle 2*pi*u2. */
void or_box_muller(double u1, double u2, double *z0, double *z1)
{
    double r = sqrt(-2.0 * log(u1));
    double th = 2.0 * M_PI * u2;
    *z0 = r * cos(th);
    *z1 = r * sin(th);
}

/* Uniform-discrete on {lo..hi} from one word: lo + floor(w * (hi-lo+1) / 2^32). */
int64_t or_uniform_discrete(uint32_t w, int64_t lo, int64_t hi)
{
    uint64_t range = (uint64_t)(hi - lo + 1);
    return lo + (int64_t)(((uint64_t)w * range) >> 32);
}

/* Four single-precision-stream normals from one Philox block (two Box-Muller pairs). */
static void normals4_single(const uint32_t w[4], double z[4])
{
    or_box_muller(or_u01_single(w[0]), or_u01_single(w[1]), &z[0], &z[1]);
    or_box_muller(or_u01_single(w[2]), or_u01_single(w[3]), &z[2], &z[3]);
}

/* ---------------------------------------------------- compensated sums -- */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(nsum a) { return a.s + a.c; }

/* ------------------------------------------------- log-sum-exp and ESS -- */
/* out = {max, s1 = sum exp(l-m), s2 = sum exp(2(l-m)), LSE = m + log s1, ESS = s1^2/s2}.
 * -inf entries contribute zero.  All entries -inf: LSE = -inf, ESS = 0. */
void or_lse_ess(const double *lw, int64_t n, double out[5])
{
    double m = -INFINITY;
    for (int64_t i = 0; i < n; ++i) if (lw[i] > m) m = lw[i];
    if (!(m > -INFINITY)) {
        out[0] = m; out[1] = 0.0; out[2] = 0.0; out[3] = -INFINITY; out[4] = 0.0;
        return;
    }
    nsum s1 = {0, 0}, s2 = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        double e = exp(lw[i] - m);
        nadd(&s1, e);
        nadd(&s2, e * e);
    }
    double a = nval(s1), b = nval(s2);
    out[0] = m; out[1] = a; out[2] = b; out[3] = m + log(a); out[4] = a * a / b;
}

/* ------------------------------------------------------------- models -- */
enum { MODEL_POLY = 1, MODEL_BLR = 2, MODEL_LGSSM = 3, MODEL_GMM = 4 };

/* POLY (paper Sec. 1.1): n ~ UniformDiscrete{2..5}; c_j ~ Normal(0, sd), j < n;
 * factor(-sum_d (y_d - poly_c(x_d))^2 / 2).  Word allocation per particle i:
 * block 0 word 0 -> n; blocks 1..3 -> one double-precision Box-Muller pair each,
 * giving c_0..c_5 (always all drawn; only c_0..c_{n-1} are used).
 * hyper = {sd, n_lo, n_hi}. */
void or_poly_draw(uint64_t seed, int64_t i, uint32_t tag, const double *hyper,
                  int32_t *n_out, double c[6])
{
    uint32_t w[4];
    draw4(seed, (uint32_t)i, 0, 0, 0, tag, w);
    *n_out = (int32_t)or_uniform_discrete(w[0], (int64_t)hyper[1], (int64_t)hyper[2]);
    for (uint32_t b = 1; b <= 3; ++b) {
        draw4(seed, (uint32_t)i, b, 0, 0, tag, w);
        double z0, z1;
        or_box_muller(or_u01_double(w[0], w[1]), or_u01_double(w[2], w[3]), &z0, &z1);
        c[2 * (b - 1)] = hyper[0] * z0;
        c[2 * (b - 1) + 1] = hyper[0] * z1;
    }
}

/* Horner over c_{n-1}..c_0, then -1/2 * sum of squared residuals. */
double or_poly_loglik(int32_t n, const double *c, const double *x, const double *y, int64_t D)
{
    double acc = 0.0;
    for (int64_t d = 0; d < D; ++d) {
        double p = 0.0;
        for (int32_t j = n - 1; j >= 0; --j) p = p * x[d] + c[j];
        double r = y[d] - p;
        acc += r * r;
    }
    return -0.5 * acc;
}

/* BLR: w_k ~ Normal(0, prior_sd), k < d (d <= 16, multiple of 4);
 * observe(Normal(x_d . w, noise_sd), y_d) for every row d.
 * Word allocation: block b gives w_{4b..4b+3} (two single-precision Box-Muller pairs).
 * hyper = {prior_sd, noise_sd}. */
void or_blr_draw_std(uint64_t seed, int64_t i, uint32_t tag, int32_t dim, double z[16])
{
    uint32_t w[4];
    for (int32_t b = 0; b < dim / 4; ++b) {
        draw4(seed, (uint32_t)i, (uint32_t)b, 0, 0, tag, w);
        normals4_single(w, z + 4 * b);
    }
}

double or_blr_loglik(const double *wv, int32_t dim, const double *X, const double *y,
                     int64_t D, double noise_sd)
{
    double var = noise_sd * noise_sd;
    double c = -0.5 * log(2.0 * M_PI * var);
    double acc = 0.0;
    for (int64_t d = 0; d < D; ++d) {
        double mu = 0.0;
        for (int32_t k = 0; k < dim; ++k) mu += X[d * dim + k] * wv[k];
        double r = y[d] - mu;
        acc += c - r * r / (2.0 * var);
    }
    return acc;
}

/* Gaussian proposal q = N(mean, L L^T) for BLR (L lower-triangular, row-major).
 * w = mean + L z with z standard normal from the PROPOSAL stream; returns
 * log p(w) - log q(w) where p is the N(0, prior_sd^2 I) prior. */
static double blr_proposal_draw(uint64_t seed, int64_t i, int32_t dim, const double *qp,
                                double prior_sd, double wv[16])
{
    double z[16];
    or_blr_draw_std(seed, i, TAG_PROPOSAL, dim, z);
    const double *mean = qp, *L = qp + dim;
    double logdet = 0.0, zz = 0.0, ww = 0.0;
    for (int32_t r = 0; r < dim; ++r) {
        double v = mean[r];
        for (int32_t k = 0; k <= r; ++k) v += L[r * dim + k] * z[k];
        wv[r] = v;
        logdet += log(L[r * dim + r]);
        zz += z[r] * z[r];
        ww += v * v;
    }
    double log_q = -0.5 * zz - logdet - 0.5 * dim * log(2.0 * M_PI);
    double log_p = -0.5 * ww / (prior_sd * prior_sd) - dim * log(prior_sd) - 0.5 * dim * log(2.0 * M_PI);
    return log_p - log_q;
}

/* ------------------------------------------------- importance sampling -- */
/* Summary layout.
 *   POLY: [0..3]  P(n = 2..5 | y)
 *         [4..23] E[c_j | n, y] for n = 2..5 (5 slots each, zero beyond n; zero if mass 0)
 *         [24..28] E[c_j 1{j < n} | y] (zero-padded marginal)          -> 29 values
 *   BLR:  [0..d-1] E[w | y]                                             -> d values
 * scalars = {log Z-hat, ESS, max lw, s1, s2}. */
int or_importance(int32_t model, const double *x, const double *y, int64_t D, int32_t dim,
                  const double *hyper, int64_t N, uint64_t seed,
                  int32_t q_kind, const double *q_params,
                  double *lw_out, double *lat_out, double *summaries, double *scalars)
{
    if (N <= 0) return -1;
    if (model != MODEL_POLY && model != MODEL_BLR) return -2;
    if (model == MODEL_BLR && (dim <= 0 || dim > 16 || dim % 4)) return -1;
    int n_lat = model == MODEL_POLY ? 6 : dim;       /* POLY: n plus c_0..c_4 */
    double *lw = (double *)malloc(sizeof(double) * N);
    double *lat = (double *)malloc(sizeof(double) * N * n_lat);
    if (!lw || !lat) { free(lw); free(lat); return -3; }

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if (model == MODEL_POLY) {
            int32_t n; double c[6];
            or_poly_draw(seed, i, TAG_PRIOR, hyper, &n, c);
            lw[i] = or_poly_loglik(n, c, x, y, D);
            lat[0 * N + i] = n;
            for (int j = 0; j < 5; ++j) lat[(1 + j) * N + i] = c[j];
        } else {
            double wv[16], extra = 0.0;
            if (q_kind == 1) {
                extra = blr_proposal_draw(seed, i, dim, q_params, hyper[0], wv);
            } else {
                double z[16];
                or_blr_draw_std(seed, i, TAG_PRIOR, dim, z);
                for (int k = 0; k < dim; ++k) wv[k] = hyper[0] * z[k];
            }
            lw[i] = or_blr_loglik(wv, dim, x, y, D, hyper[1]) + extra;
            for (int k = 0; k < dim; ++k) lat[k * N + i] = wv[k];
        }
    }

    double st[5];
    or_lse_ess(lw, N, st);
    scalars[0] = st[3] - log((double)N);
    scalars[1] = st[4];
    scalars[2] = st[0];
    scalars[3] = st[1];
    scalars[4] = st[2];

    if (summaries) {
        double m = st[0];
        if (model == MODEL_POLY) {
            nsum mass[4] = {{0}}, cm[4][5] = {{{0}}}, marg[5] = {{0}};
            for (int64_t i = 0; i < N; ++i) {
                double e = exp(lw[i] - m);
                int n = (int)lat[i];
                nadd(&mass[n - 2], e);
                for (int j = 0; j < n; ++j) {
                    double c = lat[(1 + j) * N + i];
                    nadd(&cm[n - 2][j], e * c);
                    nadd(&marg[j], e * c);
                }
            }
            for (int k = 0; k < 4; ++k) {
                double mk = nval(mass[k]);
                summaries[k] = mk / st[1];
                for (int j = 0; j < 5; ++j)
                    summaries[4 + 5 * k + j] = mk > 0 ? nval(cm[k][j]) / mk : 0.0;
            }
            for (int j = 0; j < 5; ++j) summaries[24 + j] = nval(marg[j]) / st[1];
        } else {
            for (int k = 0; k < dim; ++k) {
                nsum a = {0, 0};
                for (int64_t i = 0; i < N; ++i) nadd(&a, exp(lw[i] - m) * lat[k * N + i]);
                summaries[k] = nval(a) / st[1];
            }
        }
    }
    if (lw_out) memcpy(lw_out, lw, sizeof(double) * N);
    if (lat_out) memcpy(lat_out, lat, sizeof(double) * N * n_lat);
    free(lw); free(lat);
    return 0;
}

/* Per-particle log-weights for an arbitrary list of particle indices (used to
 * check sampled outputs of a full-size run one particle at a time). */
int or_particle_logweights(int32_t model, const double *x, const double *y, int64_t D,
                           int32_t dim, const double *hyper, uint64_t seed,
                           int32_t q_kind, const double *q_params,
                           int64_t m, const int64_t *idx, double *lw, double *lat /* [m][6 or dim] */)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = idx[r];
        if (model == MODEL_POLY) {
            int32_t n; double c[6];
            or_poly_draw(seed, i, TAG_PRIOR, hyper, &n, c);
            lw[r] = or_poly_loglik(n, c, x, y, D);
            if (lat) { lat[r * 6] = n; for (int j = 0; j < 5; ++j) lat[r * 6 + 1 + j] = c[j]; }
        } else {
            double wv[16], extra = 0.0;
            if (q_kind == 1) extra = blr_proposal_draw(seed, i, dim, q_params, hyper[0], wv);
            else {
                double z[16];
                or_blr_draw_std(seed, i, TAG_PRIOR, dim, z);
                for (int k = 0; k < dim; ++k) wv[k] = hyper[0] * z[k];
            }
            lw[r] = or_blr_loglik(wv, dim, x, y, D, hyper[1]) + extra;
            if (lat) for (int k = 0; k < dim; ++k) lat[r * dim + k] = wv[k];
        }
    }
    return 0;
}

/* ------------------------------------------------------------ resampling -- */
/* Quantisation exponent: q_i = floor(exp(lw_i - max) * 2^k), k = 62 - ceil(log2 N),
 * so that the total S = sum q_i fits in 62 bits. */
int32_t or_quant_bits(int64_t N)
{
    int c = 0;
    while (((int64_t)1 << c) < N) ++c;
    return 62 - c;
}

/* Systematic resampling with integer-quantised weights (association-free).
 *   Q = inclusive prefix sum of q, S = Q_{N-1};
 *   R = one 64-bit word (words 0,1 of block (0, 0, step, inst<<8 | RESAMPLE));
 *   U = floor(R * S / 2^64);  ancestor a(j) = min{a : N * Q_a > j * S + U}.
 * tie (optional): slot j is flagged when the slot point j*S+U lies within
 * band * N * S of either neighbouring boundary N*Q_{a-1}, N*Q_a.
 * Returns 0, or -1 when no weight is positive (every entry -inf or NaN). */
int or_resample(const double *lw, int64_t N, uint64_t seed, uint32_t step, uint32_t inst,
                int32_t *anc, double band, uint8_t *tie)
{
    double m = -INFINITY;
    for (int64_t i = 0; i < N; ++i) if (lw[i] > m) m = lw[i];
    if (!(m > -INFINITY)) return -1;
    int32_t k = or_quant_bits(N);
    uint64_t *Q = (uint64_t *)malloc(sizeof(uint64_t) * N);
    if (!Q) return -3;
    uint64_t acc = 0;
    for (int64_t i = 0; i < N; ++i) {
        double e = exp(lw[i] - m);
        uint64_t q = (uint64_t)floor(ldexp(e, k));
        acc += q;
        Q[i] = acc;
    }
    uint64_t S = acc;
    uint32_t w[4];
    draw4(seed, 0, 0, step, inst, TAG_RESAMPLE, w);
    uint64_t R = ((uint64_t)w[1] << 32) | w[0];
    uint64_t U = (uint64_t)(((unsigned __int128)R * S) >> 64);
    long double tot = (long double)N * (long double)S;
    int64_t a = 0;
    for (int64_t j = 0; j < N; ++j) {
        unsigned __int128 t = (unsigned __int128)j * S + U;
        while ((unsigned __int128)N * Q[a] <= t) ++a;
        anc[j] = (int32_t)a;
        if (tie) {
            unsigned __int128 hi = (unsigned __int128)N * Q[a];
            unsigned __int128 lo = a > 0 ? (unsigned __int128)N * Q[a - 1] : 0;
            long double d1 = (long double)(hi - t), d2 = (long double)(t - lo);
            long double dm = d1 < d2 ? d1 : d2;
            tie[j] = (uint8_t)(dm <= (long double)band * tot);
        }
    }
    free(Q);
    return 0;
}

/* Textbook FP64 systematic resampling with the same uniform u = R / 2^64:
 * a(j) = min{a : C_a > (j + u) / N}, C = cumulative normalised weights. */
int or_resample_textbook(const double *lw, int64_t N, uint64_t seed, uint32_t step,
                         uint32_t inst, int32_t *anc)
{
    double m = -INFINITY;
    for (int64_t i = 0; i < N; ++i) if (lw[i] > m) m = lw[i];
    if (!(m > -INFINITY)) return -1;
    double *C = (double *)malloc(sizeof(double) * N);
    if (!C) return -3;
    nsum s = {0, 0};
    for (int64_t i = 0; i < N; ++i) { nadd(&s, exp(lw[i] - m)); C[i] = nval(s); }
    double tot = C[N - 1];
    uint32_t w[4];
    draw4(seed, 0, 0, step, inst, TAG_RESAMPLE, w);
    double u = (double)(((uint64_t)w[1] << 32) | w[0]) * 0x1p-64;
    int64_t a = 0;
    for (int64_t j = 0; j < N; ++j) {
        double p = (j + u) / (double)N;
        while (a < N - 1 && C[a] / tot <= p) ++a;
        anc[j] = (int32_t)a;
    }
    free(C);
    return 0;
}

/* ------------------------------------------------------------------ SMC -- */
/* LGSSM (bootstrap filter):  x_0 = m0 + p0_sd * z;  x_s = a x_{s-1} + q_sd eps_s;
 * observe(Normal(x_s, r_sd), y_s).  hyper = {a, q_sd, r_sd, m0, p0_sd}.
 * Noise word allocation for slot i: eps_s = the (s mod 4)-th normal of block
 * (i, 0, s div 4, PRIOR) (two single-precision Box-Muller pairs); the initial
 * normal is normal 0 of block (i, 1, 0, PRIOR).
 *
 * GMM (mixture with known K, unit-sd components by default): pi ~ Dirichlet(1_K)
 * as normalised Exp(1) draws E_k = -ln u (words 0..7 of blocks 0,1), mu_k ~
 * Normal(0, mu_sd) (normals 0..7 of blocks 2,3); one factor per datum,
 * log sum_k pi_k Normal(y_s; mu_k, comp_sd).  hyper = {mu_sd, comp_sd}.
 * State layout [field][N]: GMM fields 0..K-1 = log pi_k, K..2K-1 = mu_k. */
static inline void lgssm_eps4(uint64_t seed, int64_t i, uint32_t grp, uint32_t inst, double z[4])
{
    uint32_t w[4];
    draw4(seed, (uint32_t)i, 0, grp, inst, TAG_PRIOR, w);
    normals4_single(w, z);
}

static void gmm_init_particle(uint64_t seed, int64_t i, uint32_t inst, int32_t K,
                              const double *hyper, double *lpi, double *mu)
{
    uint32_t w[8];
    draw4(seed, (uint32_t)i, 0, 0, inst, TAG_PRIOR, w);
    draw4(seed, (uint32_t)i, 1, 0, inst, TAG_PRIOR, w + 4);
    double E[8], tot = 0.0;
    for (int k = 0; k < K; ++k) { E[k] = -log(or_u01_single(w[k])); tot += E[k]; }
    for (int k = 0; k < K; ++k) lpi[k] = log(E[k] / tot);
    double z[8];
    uint32_t v[4];
    draw4(seed, (uint32_t)i, 2, 0, inst, TAG_PRIOR, v);
    normals4_single(v, z);
    draw4(seed, (uint32_t)i, 3, 0, inst, TAG_PRIOR, v);
    normals4_single(v, z + 4);
    for (int k = 0; k < K; ++k) mu[k] = hyper[0] * z[k];
}

/* log sum_k pi_k Normal(y; mu_k, sd), evaluated with the max shift. */
double or_gmm_logfactor(int32_t K, const double *lpi, const double *mu, double sd, double y)
{
    double t[8], mx = -INFINITY;
    double c = -0.5 * log(2.0 * M_PI) - log(sd);
    for (int k = 0; k < K; ++k) {
        double r = (y - mu[k]) / sd;
        t[k] = lpi[k] + c - 0.5 * r * r;
        if (t[k] > mx) mx = t[k];
    }
    if (!(mx > -INFINITY)) return -INFINITY;
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += exp(t[k] - mx);
    return mx + log(s);
}

/* Initial particle states, layout [field][N] (see the model notes above). */
static void smc_init_state(int32_t model, int32_t K, const double *hyper, int64_t N, uint64_t seed,
                           uint32_t inst, double *st)
{
    if (model == MODEL_LGSSM) {
        for (int64_t i = 0; i < N; ++i) {
            double z0 = 0.0;
            if (hyper[4] != 0.0) {
                uint32_t w[4]; double z[4];
                draw4(seed, (uint32_t)i, 1, 0, inst, TAG_PRIOR, w);
                normals4_single(w, z);
                z0 = z[0];
            }
            st[i] = hyper[3] + hyper[4] * z0;
        }
    } else {
        for (int64_t i = 0; i < N; ++i) {
            double lpi[8], mu[8];
            gmm_init_particle(seed, i, inst, K, hyper, lpi, mu);
            for (int k = 0; k < K; ++k) { st[k * N + i] = lpi[k]; st[(K + k) * N + i] = mu[k]; }
        }
    }
}

/* Factor s: every particle moves to step s (LGSSM) and adds its log-factor. */
static void smc_advance(int32_t model, int32_t K, const double *hyper, const double *y, int64_t s,
                        int64_t N, uint64_t seed, uint32_t inst, double *st, double *lw)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if (model == MODEL_LGSSM) {
            double z[4];
            lgssm_eps4(seed, i, (uint32_t)(s >> 2), inst, z);
            double xv = hyper[0] * st[i] + hyper[1] * z[s & 3];
            st[i] = xv;
            double r = (y[s] - xv) / hyper[2];
            lw[i] += -0.5 * log(2.0 * M_PI) - log(hyper[2]) - 0.5 * r * r;
        } else {
            double lpi[8], mu[8];
            for (int k = 0; k < K; ++k) { lpi[k] = st[k * N + i]; mu[k] = st[(K + k) * N + i]; }
            lw[i] += or_gmm_logfactor(K, lpi, mu, hyper[1], y[s]);
        }
    }
}

/* ------------------------------------------------- enumeration (HMM) -- */
/* Exact inference by enumeration (paper Sec. 3.6.1): every execution of a
 * model whose sample sites all have finite support, each weighted by the
 * product of its sample probabilities and factors.  Model: a hidden Markov
 * chain of K states over T steps, z_0 ~ Cat(pi0), z_t ~ Cat(A[z_{t-1}]),
 * observe(Normal(mu[z_t], sigma), y_t).  An execution is a path z; its
 * index is sum_t z_t K^(T-1-t).  hyper = {K, sigma, pi0[K], A[K][K]
 * (row = from), mu[K]}.  Outputs: scal[4] = {log Z, paths, log joint of the
 * MAP path, 0}; marg[T][K] = P(z_t = k | y); map[T] the most probable path
 * (the lowest index among equals).  Plain: the paths in index order, the
 * log-sum-exp with compensated sums (max first).  Returns -1 on bad
 * arguments, -3 on allocation failure. */
static double hmm_path_lw(int32_t K, int64_t T, const double *lpi, const double *lA, const double *y,
                          const double *mu, double sigma, const int32_t *z)
{
    double lw = lpi[z[0]];
    for (int64_t t = 0; t < T; ++t) {
        if (t > 0) lw += lA[z[t - 1] * K + z[t]];
        double r = (y[t] - mu[z[t]]) / sigma;
        lw += -0.5 * log(2.0 * M_PI) - log(sigma) - 0.5 * r * r;
    }
    return lw;
}

int or_enumerate_hmm(const double *y, int64_t T, const double *hyper, double *scal, double *marg, int32_t *map)
{
    int32_t K = (int32_t)hyper[0];
    if (K < 1 || K > 8 || T < 1 || T > 40) return -1;
    double paths = pow((double)K, (double)T);
    if (paths > 4e12) return -1;
    double sigma = hyper[1];
    const double *pi0 = hyper + 2, *A = hyper + 2 + K, *mu = hyper + 2 + K + K * K;
    double lpi[8], lA[64];
    for (int k = 0; k < K; ++k) lpi[k] = log(pi0[k]);
    for (int k = 0; k < K * K; ++k) lA[k] = log(A[k]);
    int64_t P = (int64_t)paths;
    /* pass 1: the largest log-weight and the MAP path */
    double m = -INFINITY;
    int64_t best = 0;
#pragma omp parallel
    {
        double ml = -INFINITY;
        int64_t bl = 0;
        int32_t z[40];
#pragma omp for schedule(static)
        for (int64_t p = 0; p < P; ++p) {
            int64_t q = p;
            for (int64_t t = T - 1; t >= 0; --t) { z[t] = (int32_t)(q % K); q /= K; }
            double lw = hmm_path_lw(K, T, lpi, lA, y, mu, sigma, z);
            if (lw > ml) { ml = lw; bl = p; }
        }
#pragma omp critical
        { if (ml > m || (ml == m && bl < best)) { m = ml; best = bl; } }
    }
    /* pass 2: sums of exp(lw - m), overall and per (t, k) */
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *part = (double *)calloc((size_t)nth * (1 + T * K), sizeof(double));
    if (!part) return -3;
#pragma omp parallel
    {
        int th = 0;
#ifdef _OPENMP
        th = omp_get_thread_num();
#endif
        double *mine = part + (size_t)th * (1 + T * K);
        int32_t z[40];
        /* static schedule: thread th takes one contiguous range of paths, in order */
#pragma omp for schedule(static)
        for (int64_t p = 0; p < P; ++p) {
            int64_t q = p;
            for (int64_t t = T - 1; t >= 0; --t) { z[t] = (int32_t)(q % K); q /= K; }
            double e = exp(hmm_path_lw(K, T, lpi, lA, y, mu, sigma, z) - m);
            mine[0] += e;
            for (int64_t t = 0; t < T; ++t) mine[1 + t * K + z[t]] += e;
        }
    }
    double tot[1 + 40 * 8];
    for (int64_t f = 0; f < 1 + T * K; ++f) {
        nsum a = {0, 0};
        for (int th = 0; th < nth; ++th) nadd(&a, part[(size_t)th * (1 + T * K) + f]);
        tot[f] = nval(a);
    }
    free(part);
    if (scal) {
        scal[0] = m + log(tot[0]);
        scal[1] = paths;
        scal[2] = m;
        scal[3] = 0.0;
    }
    if (marg) for (int64_t f = 0; f < T * K; ++f) marg[f] = tot[1 + f] / tot[0];
    if (map) {
        int64_t q = best;
        for (int64_t t = T - 1; t >= 0; --t) { map[t] = (int32_t)(q % K); q /= K; }
    }
    return 0;
}

/* ----------------------------------------- lightweight MH (POLY model) -- */
/* Lightweight Metropolis-Hastings (paper Sec. 3.6.3) on the polynomial model,
 * many independent chains.  A chain's trace holds the sites the execution
 * reached: n and c_0..c_{n-1} (n + 1 sites).  One iteration picks a site of
 * the trace uniformly, resamples it from its prior and re-executes: when n
 * changes, the coefficients both executions reach keep their values, those
 * only the new one reaches are drawn fresh from their prior, and those only
 * the old one reached are dropped.  With prior proposals every prior density
 * cancels, and the acceptance ratio is
 *     alpha = L(x') / L(x) * (n + 1) / (n' + 1)
 * (the likelihood ratio times the ratio of the site counts).
 *
 * Words of iteration t of chain c (tag 8): block (c, 3t, 0) word 0 picks the
 * site (uniform discrete over 0..n; 0 is n, j + 1 is c_j), word 1 the
 * proposed n' (uniform discrete over n_lo..n_hi), word 2 the acceptance
 * uniform v (single-precision stream); blocks (c, 3t + 1, 0) and (c, 3t + 2, 0)
 * give one double-precision Box-Muller pair each, z_0..z_3: a resampled c_j is
 * sd z_0, fresh coefficients c_n, c_{n+1}, ... are sd z_1, sd z_2, sd z_3.
 * The chain starts from the prior draw of the importance sampler (particle c);
 * unused coefficient slots hold 0.  Accepted when log v < log alpha. */
#define TAG_MCMC 8

/* One chain.  Outputs per iteration (optional): n_tr[t], la_tr[t] (log alpha).
 * g_la (optional): the other run's log alpha per iteration; where
 * |log alpha - log v| <= 2 |g_la - log alpha| + 1e-9 (1 + |l(x)|) the other
 * run's decision (log v < g_la) is taken (a tie).  st[5] and acc return the
 * chain's final coefficients and accepted count; sums[29] accumulate, over
 * iterations t >= burn_in: [n - 2] += 1, [4 + 5 (n - 2) + j] += c_j,
 * [24 + j] += c_j 1{j < n}.  tstats[3]: {ties, adopted, non-tie differences}. */
static void mcmc_chain(const double *x, const double *y, int64_t D, const double *hyper, int64_t c,
                       int64_t n_iters, int64_t burn_in, uint64_t seed, int32_t *n_io, double *st, int64_t *acc,
                       double *sums, int8_t *n_tr, double *la_tr, const double *g_la, int64_t stride,
                       int64_t *tstats)
{
    int32_t n = *n_io;
    double ll = or_poly_loglik(n, st, x, y, D);
    for (int64_t t = 0; t < n_iters; ++t) {
        uint32_t w[4], b1[4], b2[4];
        draw4(seed, (uint32_t)c, (uint32_t)(3 * t), 0, 0, TAG_MCMC, w);
        draw4(seed, (uint32_t)c, (uint32_t)(3 * t + 1), 0, 0, TAG_MCMC, b1);
        draw4(seed, (uint32_t)c, (uint32_t)(3 * t + 2), 0, 0, TAG_MCMC, b2);
        double z[4];
        or_box_muller(or_u01_double(b1[0], b1[1]), or_u01_double(b1[2], b1[3]), &z[0], &z[1]);
        or_box_muller(or_u01_double(b2[0], b2[1]), or_u01_double(b2[2], b2[3]), &z[2], &z[3]);
        int64_t site = or_uniform_discrete(w[0], 0, n);
        double c2[5];
        for (int j = 0; j < 5; ++j) c2[j] = st[j];
        int32_t n2 = n;
        if (site == 0) {
            n2 = (int32_t)or_uniform_discrete(w[1], (int64_t)hyper[1], (int64_t)hyper[2]);
            for (int32_t j = n; j < n2; ++j) c2[j] = hyper[0] * z[1 + (j - n)];
            for (int32_t j = n2; j < 5; ++j) c2[j] = 0.0;
        } else {
            c2[site - 1] = hyper[0] * z[0];
        }
        double ll2 = or_poly_loglik(n2, c2, x, y, D);
        double la = (ll2 - ll) + (log((double)(n + 1)) - log((double)(n2 + 1)));
        double lv = log(or_u01_single(w[2]));
        int a = lv < la;
        if (g_la) {
            double ga = g_la[t * stride + c];
            double dv = fabs(ga - la);
            int given = lv < ga;
            if (fabs(la - lv) <= 2.0 * dv + 1e-9 * (1.0 + fabs(ll))) {
                ++tstats[0];
                if (given != a) ++tstats[1];
                a = given;
            } else if (given != a) {
                ++tstats[2];
            }
        }
        if (la_tr) la_tr[t * stride + c] = la;
        if (a) {
            n = n2;
            for (int j = 0; j < 5; ++j) st[j] = c2[j];
            ll = ll2;
            ++*acc;
        }
        if (n_tr) n_tr[t * stride + c] = (int8_t)n;
        if (t >= burn_in && sums) {
            sums[n - 2] += 1.0;
            for (int j = 0; j < n; ++j) { sums[4 + 5 * (n - 2) + j] += st[j]; sums[24 + j] += st[j]; }
        }
    }
    *n_io = n;
}

/* n_chains chains of n_iters iterations each.  Outputs (any may be NULL):
 * state_out[6][n_chains] final n and c_0..c_4 (unused slots 0); accepts
 * [n_chains]; summaries[29] over all chains' iterations t >= burn_in: P(n | y)
 * for n = 2..5, E[c_j | n, y] (0 where n has no mass), E[c_j 1{j < n} | y]
 * (the layout of importance sampling); n_trace / la_trace [n_iters][n_chains];
 * g_la [n_iters][n_chains] and tstats[3] for a forced run beside another.
 * Returns 0 or -1 on bad arguments, -3 on allocation failure. */
int or_mcmc_poly(const double *x, const double *y, int64_t D, const double *hyper, int64_t n_chains, int64_t n_iters,
                 int64_t burn_in, uint64_t seed, double *state_out, int64_t *accepts, double *summaries,
                 int8_t *n_trace, double *la_trace, const double *g_la, int64_t *tstats)
{
    if (n_chains <= 0 || n_iters < 0 || burn_in < 0 || D < 0) return -1;
    if (hyper[1] < 1 || hyper[2] > 5 || hyper[1] > hyper[2]) return -1;
    double *sums = (double *)calloc((size_t)n_chains * 29, sizeof(double));
    if (!sums) return -3;
    int64_t ties = 0, adopted = 0, bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+:ties, adopted, bad)
    for (int64_t c = 0; c < n_chains; ++c) {
        int32_t n;
        double cc[6];
        or_poly_draw(seed, c, TAG_PRIOR, hyper, &n, cc);
        for (int j = n; j < 5; ++j) cc[j] = 0.0;
        int64_t acc = 0, ts[3] = {0, 0, 0};
        mcmc_chain(x, y, D, hyper, c, n_iters, burn_in, seed, &n, cc, &acc, sums + (size_t)c * 29, n_trace, la_trace,
                   g_la, n_chains, ts);
        ties += ts[0]; adopted += ts[1]; bad += ts[2];
        if (state_out) {
            state_out[c] = (double)n;
            for (int j = 0; j < 5; ++j) state_out[(size_t)(1 + j) * n_chains + c] = cc[j];
        }
        if (accepts) accepts[c] = acc;
    }
    if (summaries) {
        double tot[29];
        for (int k = 0; k < 29; ++k) {
            nsum a = {0, 0};
            for (int64_t c = 0; c < n_chains; ++c) nadd(&a, sums[(size_t)c * 29 + k]);
            tot[k] = nval(a);
        }
        double all = tot[0] + tot[1] + tot[2] + tot[3];
        for (int m = 0; m < 4; ++m) {
            summaries[m] = all > 0 ? tot[m] / all : 0.0;
            for (int j = 0; j < 5; ++j) summaries[4 + 5 * m + j] = tot[m] > 0 ? tot[4 + 5 * m + j] / tot[m] : 0.0;
        }
        for (int j = 0; j < 5; ++j) summaries[24 + j] = all > 0 ? tot[24 + j] / all : 0.0;
    }
    if (tstats) { tstats[0] = ties; tstats[1] = adopted; tstats[2] = bad; }
    free(sums);
    return 0;
}

/* ------------------------------------------------ resample-move (GMM) -- */
/* Resample-move: after each resampling at factor s the mixture particles take
 * M Metropolis-Hastings steps whose target is the posterior given the data
 * seen so far, p(theta) prod_{d <= s} f(y_d | theta) -- particle inference
 * (named as future work in Sec. 6) with the Metropolis-Hastings acceptance
 * rule of the paper's third inference method (Sec. 3.6.3).  The move leaves
 * the equally weighted population's target invariant, so log-weights stay 0.
 *
 * Readings (the paper gives no move kernel):
 *   - unconstrained coordinates u = (b_1..b_{K-1}, mu_1..mu_K) with
 *     b_k = log pi_k - log pi_K; log pi_k = b_k - log(1 + sum_j e^{b_j});
 *   - prior density of u: Dirichlet(1) gives log (K-1)! + sum_k log pi_k (the
 *     softmax Jacobian), plus sum_k log Normal(mu_k; 0, mu_sd);
 *   - Gaussian random walk u' = u + h z, symmetric, with scales fixed by s:
 *     h_mu = lam / sqrt(1/mu_sd^2 + (s+1)/(K comp_sd^2)),
 *     h_b  = lam / sqrt(3/pi^2 + (s+1)/(2K))
 *     (the posterior sds if each component held (s+1)/K of the data; pi^2/3
 *     is the prior variance of b_k), lam = 2.38 / sqrt(2K - 1) unless given;
 *   - accept when log v < log alpha = [l(u') + log p(u')] - [l(u) + log p(u)],
 *     l the log-likelihood of y_0..y_s;
 *   - words: move m of slot j at factor s uses Philox blocks
 *     (j, 8m + b, s, inst << 8 | 7): blocks b = 0..3 give 16 normals
 *     (single-precision Box-Muller pairs, the first 2K - 1 used), word 0 of
 *     block 4 the uniform v. */
#define TAG_MOVE 7

static double gmm_loglik_upto(int32_t K, const double *lpi, const double *mu, double sd, const double *y, int64_t s)
{
    double l = 0.0;
    for (int64_t d = 0; d <= s; ++d) l += or_gmm_logfactor(K, lpi, mu, sd, y[d]);
    return l;
}

static double gmm_log_prior(int32_t K, const double *lpi, const double *mu, double mu_sd)
{
    double l = 0.0;
    for (int k = 0; k < K; ++k) l += lpi[k] - 0.5 * (mu[k] / mu_sd) * (mu[k] / mu_sd);
    return l;           /* constants (log (K-1)!, the normal's) cancel in the ratio */
}

void or_move_scales(int32_t K, int64_t s, const double *hyper, double lam, double *h_b, double *h_mu)
{
    if (!(lam > 0.0)) lam = 2.38 / sqrt(2.0 * K - 1.0);
    double n = (double)(s + 1);
    *h_mu = lam / sqrt(1.0 / (hyper[0] * hyper[0]) + n / ((double)K * hyper[1] * hyper[1]));
    *h_b = lam / sqrt(3.0 / (M_PI * M_PI) + n / (2.0 * K));
}

/* One particle's proposal for move m: u' = u + h z, mapped back to (log pi, mu). */
static void gmm_move_propose(uint64_t seed, int64_t j, int m, int64_t s, uint32_t inst, int32_t K, double h_b,
                             double h_mu, const double *lpi, const double *mu, double *lpi2, double *mu2,
                             double *logv)
{
    uint32_t w[4];
    double z[16];
    for (int b = 0; b < 4; ++b) {
        draw4(seed, (uint32_t)j, (uint32_t)(8 * m + b), (uint32_t)s, inst, TAG_MOVE, w);
        normals4_single(w, z + 4 * b);
    }
    draw4(seed, (uint32_t)j, (uint32_t)(8 * m + 4), (uint32_t)s, inst, TAG_MOVE, w);
    *logv = log(or_u01_single(w[0]));
    double b2[8], mx = 0.0;
    for (int k = 0; k < K - 1; ++k) {
        b2[k] = (lpi[k] - lpi[K - 1]) + h_b * z[k];
        if (b2[k] > mx) mx = b2[k];
    }
    double se = exp(-mx);                    /* the fixed coordinate b_K = 0 */
    for (int k = 0; k < K - 1; ++k) se += exp(b2[k] - mx);
    double lse = mx + log(se);
    for (int k = 0; k < K - 1; ++k) lpi2[k] = b2[k] - lse;
    lpi2[K - 1] = -lse;
    for (int k = 0; k < K; ++k) mu2[k] = mu[k] + h_mu * z[K - 1 + k];
}

/* M moves of every particle after the resampling at factor s (state
 * [2K][N], see the model notes).  alpha_out[M][N] (optional): this run's
 * log alpha.  Forcing (g_alpha non-NULL, [M][N], the other run's FP64
 * log alpha): where |log alpha - log v| <= 2 |g_alpha - log alpha| + 1e-12
 * (1 + |log alpha|) the decision is a tie and the other run's decision
 * (log v < g_alpha) is adopted; elsewhere a differing decision is counted.
 * stats[4] (optional, with forcing): {tie decisions, adopted, non-tie
 * differences, max |g_alpha - log alpha| / (1 + |l(u)|)}. */
static void gmm_moves(int32_t K, const double *hyper, const double *y, int64_t s, int64_t N, uint64_t seed,
                      uint32_t inst, int32_t M, double lam, double *st, double *alpha_out, const double *g_alpha,
                      double *stats)
{
    double h_b, h_mu;
    or_move_scales(K, s, hyper, lam, &h_b, &h_mu);
    int64_t ties = 0, adopted = 0, bad = 0;
    double maxd = 0.0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+:ties, adopted, bad) reduction(max:maxd)
    for (int64_t j = 0; j < N; ++j) {
        double lpi[8], mu[8], lpi2[8], mu2[8], logv;
        for (int k = 0; k < K; ++k) { lpi[k] = st[k * N + j]; mu[k] = st[(K + k) * N + j]; }
        double ll = gmm_loglik_upto(K, lpi, mu, hyper[1], y, s);
        double lp = gmm_log_prior(K, lpi, mu, hyper[0]);
        for (int m = 0; m < M; ++m) {
            gmm_move_propose(seed, j, m, s, inst, K, h_b, h_mu, lpi, mu, lpi2, mu2, &logv);
            double ll2 = gmm_loglik_upto(K, lpi2, mu2, hyper[1], y, s);
            double lp2 = gmm_log_prior(K, lpi2, mu2, hyper[0]);
            double la = (ll2 + lp2) - (ll + lp);
            if (alpha_out) alpha_out[(size_t)m * N + j] = la;
            int acc = logv < la;
            if (g_alpha) {
                double ga = g_alpha[(size_t)m * N + j];
                double dv = fabs(ga - la);
                double rel = dv / (1.0 + fabs(ll));
                if (!(rel <= maxd)) maxd = rel;
                int given = logv < ga;
                if (fabs(la - logv) <= 2.0 * dv + 1e-12 * (1.0 + fabs(la))) {
                    ++ties;
                    if (given != acc) ++adopted;
                    acc = given;
                } else if (given != acc) {
                    ++bad;
                }
            }
            if (acc) {
                for (int k = 0; k < K; ++k) { lpi[k] = lpi2[k]; mu[k] = mu2[k]; }
                ll = ll2;
                lp = lp2;
            }
        }
        for (int k = 0; k < K; ++k) { st[k * N + j] = lpi[k]; st[(K + k) * N + j] = mu[k]; }
    }
    if (stats) { stats[0] = (double)ties; stats[1] = (double)adopted; stats[2] = (double)bad; stats[3] = maxd; }
}

/* The moves of one event applied to a given population st[2K][N] (the
 * state layout of the SMC), with this run's log alphas in alpha_out[M][N]
 * (optional): the MH kernel on its own, for the tests that pin it. */
void or_gmm_move_population(int32_t K, const double *hyper, const double *y, int64_t s, int64_t N,
                            uint64_t seed, uint32_t inst, int32_t M, double lam, double *st, double *alpha_out)
{
    gmm_moves(K, hyper, y, s, N, seed, inst, M, lam, st, alpha_out, NULL, NULL);
}

/* Generic SMC driver.
 *   y[T] observations; N particles; ess_frac threshold (resample when ESS < ess_frac*N,
 *   never after the last factor).  log Z-hat = sum over epochs of (LSE(lw) - log N).
 * Outputs (any may be NULL):
 *   scal[4]      = {log Z-hat, final ESS, number of resamplings, status}
 *   ess_tr[T]    = ESS after factor s (before any resampling)
 *   res_tr[T]    = 1 if resampled after factor s
 *   ess_tie[T]   = 1 if |ESS/N - ess_frac| <= ess_band (decision sensitive to rounding)
 *   anc_hist[max_events][N], tie_hist[max_events][N]: ancestors / tie flags per event
 *   lw_hist[max_events][N]: the log-weights each event resampled from
 *   state_out[n_fields][N], lw_out[N]: final particles and log-weights */
int or_smc(int32_t model, const double *y, int64_t T, int32_t K, const double *hyper,
           int64_t N, uint64_t seed, uint32_t inst, double ess_frac,
           double ess_band, double anc_band, int64_t max_events,
           double *scal, double *ess_tr, uint8_t *res_tr, uint8_t *ess_tie,
           int32_t *anc_hist, uint8_t *tie_hist, double *state_out, double *lw_out, double *lw_hist,
           int32_t move_steps, double move_scale, double *alpha_hist)
{
    if (N <= 0 || T < 0 || move_steps < 0) return -1;
    if (model != MODEL_LGSSM && model != MODEL_GMM) return -2;
    if (move_steps > 0 && model != MODEL_GMM) return -2;
    if (model == MODEL_GMM && (K < 1 || K > 8)) return -1;
    int nf = model == MODEL_LGSSM ? 1 : 2 * K;
    double *st = (double *)malloc(sizeof(double) * N * nf);
    double *st2 = (double *)malloc(sizeof(double) * N * nf);
    double *lw = (double *)calloc(N, sizeof(double));
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * N);
    uint8_t *tie = (uint8_t *)malloc(N);
    if (!st || !st2 || !lw || !anc || !tie) { free(st); free(st2); free(lw); free(anc); free(tie); return -3; }
    smc_init_state(model, K, hyper, N, seed, inst, st);

    nsum logz = {0, 0};
    int64_t nres = 0, ev = 0;
    double ess = (double)N, stat[5];
    int status = 0;
    for (int64_t s = 0; s < T; ++s) {
        smc_advance(model, K, hyper, y, s, N, seed, inst, st, lw);
        or_lse_ess(lw, N, stat);
        if (!(stat[0] > -INFINITY) || isnan(stat[3])) { status = -7; ess = 0.0; break; }
        ess = stat[4];
        if (ess_tr) ess_tr[s] = ess;
        if (ess_tie) ess_tie[s] = (uint8_t)(fabs(ess / (double)N - ess_frac) <= ess_band);
        int resample = (s < T - 1) && (ess < ess_frac * (double)N);
        if (res_tr) res_tr[s] = (uint8_t)resample;
        if (resample) {
            nadd(&logz, stat[3] - log((double)N));
            int rc = or_resample(lw, N, seed, (uint32_t)s, inst, anc, anc_band, tie);
            if (rc) { status = rc; break; }
            if (anc_hist && ev < max_events) memcpy(anc_hist + ev * N, anc, sizeof(int32_t) * N);
            if (tie_hist && ev < max_events) memcpy(tie_hist + ev * N, tie, N);
            if (lw_hist && ev < max_events) memcpy(lw_hist + ev * N, lw, sizeof(double) * N);
            for (int f = 0; f < nf; ++f)
                for (int64_t j = 0; j < N; ++j) st2[f * N + j] = st[f * N + anc[j]];
            double *tmp = st; st = st2; st2 = tmp;
            if (move_steps > 0)
                gmm_moves(K, hyper, y, s, N, seed, inst, move_steps, move_scale, st,
                          (alpha_hist && ev < max_events) ? alpha_hist + (size_t)ev * move_steps * N : NULL,
                          NULL, NULL);
            for (int64_t j = 0; j < N; ++j) lw[j] = 0.0;
            ++nres; ++ev;
        }
    }
    if (status == 0) {
        if (T > 0) { or_lse_ess(lw, N, stat); nadd(&logz, stat[3] - log((double)N)); ess = stat[4]; }
        else ess = (double)N;
    }
    if (scal) {
        scal[0] = status == 0 ? nval(logz) : -INFINITY;
        scal[1] = ess; scal[2] = (double)nres; scal[3] = status;
    }
    if (state_out) memcpy(state_out, st, sizeof(double) * N * nf);
    if (lw_out) memcpy(lw_out, lw, sizeof(double) * N);
    free(st); free(st2); free(lw); free(anc); free(tie);
    return status;
}

/* One teacher-forced resampling event (see or_smc_forced).  lw[N]: this run's
 * FP64 log-weights; glw[N], ganc[N]: the other run's single-precision
 * log-weights and its ancestors; step, inst: the event's Philox counter words.
 * anc[N] receives this run's ancestors with the given ones adopted at tie
 * slots.  stats[8] (optional): {unused, max mixed |glw - lw| / max(1, |lw|),
 * tie slots, adopted tie slots, non-tie differences, expected tie slots,
 * largest band, 0}.  Returns 0, -1 if no weight is positive, -3 on allocation
 * failure, -5 if a given ancestor adopted at a tie is out of range. */
int or_forced_event(const double *lw, const float *glw, const int32_t *ganc, int64_t N, uint64_t seed,
                    uint32_t step, uint32_t inst, int32_t *anc, double *stats)
{
    double m = -INFINITY;
    for (int64_t i = 0; i < N; ++i) if (lw[i] > m) m = lw[i];
    if (!(m > -INFINITY)) return -1;
    uint64_t *Q = (uint64_t *)malloc(sizeof(uint64_t) * N);
    double *band = (double *)malloc(sizeof(double) * N);
    double *wv = (double *)malloc(sizeof(double) * N);
    if (!Q || !band || !wv) { free(Q); free(band); free(wv); return -3; }
    int32_t k = or_quant_bits(N);
    uint64_t acc = 0;
    nsum W = {0, 0}, We = {0, 0}, We2 = {0, 0};
    double max_dlw = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double e = exp(lw[i] - m);
        wv[i] = e;
        acc += (uint64_t)floor(ldexp(e, k));
        Q[i] = acc;
        double d = (double)glw[i] - lw[i];
        if (e == 0.0) d = 0.0;                              /* zero weight: no influence on the CDF */
        double dm = fabs((double)glw[i] - lw[i]) / (fabs(lw[i]) > 1.0 ? fabs(lw[i]) : 1.0);
        if (!(dm <= max_dlw)) max_dlw = dm;                 /* NaN propagates */
        nadd(&W, e);
        nadd(&We, e * d);
        nadd(&We2, e * d * d);
    }
    double Wt = nval(W), Wet = nval(We), sec = nval(We2) / Wt;
    nsum Cw = {0, 0}, Ce = {0, 0};
    double max_band = 0.0, expected = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double d = wv[i] == 0.0 ? 0.0 : (double)glw[i] - lw[i];
        nadd(&Cw, wv[i]);
        nadd(&Ce, wv[i] * d);
        double C = nval(Cw) / Wt;
        double dC = (nval(Ce) - C * Wet) / Wt;
        band[i] = 2.0 * fabs(dC) + 2.0 * sec + ldexp((double)(i + 1), -k) / Wt + 1e-15;
        if (band[i] > max_band) max_band = band[i];
        expected += 2.0 * band[i] * (double)N;
    }
    uint64_t S = acc;
    uint32_t w[4];
    draw4(seed, 0, 0, step, inst, TAG_RESAMPLE, w);
    uint64_t R = ((uint64_t)w[1] << 32) | w[0];
    uint64_t U = (uint64_t)(((unsigned __int128)R * S) >> 64);
    int64_t a = 0, ties = 0, adopted = 0, bad = 0;
    int rc = 0;
    for (int64_t j = 0; j < N; ++j) {
        unsigned __int128 t = (unsigned __int128)j * S + U;
        while ((unsigned __int128)N * Q[a] <= t) ++a;
        /* slot point and the ends of its interval, in units of the total N S */
        double tn = (double)t / ((double)N * (double)S);
        double hi = (double)Q[a] / (double)S, lo = a > 0 ? (double)Q[a - 1] / (double)S : 0.0;
        int tie = (hi - tn) <= band[a] || (a > 0 && (tn - lo) <= band[a - 1]);
        if (tie) {
            ++ties;
            if (ganc[j] != (int32_t)a) ++adopted;
            if (ganc[j] < 0 || ganc[j] >= N) rc = -5;
            anc[j] = ganc[j];
        } else {
            if (ganc[j] != (int32_t)a) ++bad;
            anc[j] = (int32_t)a;
        }
    }
    if (stats) {
        stats[0] = 0.0; stats[1] = max_dlw; stats[2] = (double)ties; stats[3] = (double)adopted;
        stats[4] = (double)bad; stats[5] = expected; stats[6] = max_band; stats[7] = 0.0;
    }
    free(Q); free(band); free(wv);
    return rc;
}

/* Teacher-forced SMC: the SMC above, run beside a second (GPU) run whose
 * resampling decisions g_res[T], ancestors g_anc[E][N] and event log-weights
 * g_lw[E][N] (the single-precision weights that run resampled from) are given.
 *
 * Decisions.  Where this run's ESS lies within ess_band * N of the threshold,
 * either decision is valid and the given one is adopted; elsewhere the two
 * must agree (a disagreement is counted and the given decision is followed, so
 * the event numbering stays aligned).
 *
 * Ancestors.  This run draws its own ancestors by the integer rule from its
 * FP64 log-weights.  A slot is a tie when its point lies closer to an end of
 * its ancestor's interval than the other run's cumulative weight at that end
 * can differ from this run's.  With e_i = lw'_i - lw_i (other run minus this
 * one, W_i the normalised weights, C_a their cumulative sum) the first-order
 * change of C_a is
 *     dC_a = sum_{i<=a} W_i e_i - C_a sum_i W_i e_i,
 * and the band at end a is 2 |dC_a| plus a slack for the second-order terms
 * (2 sum_i W_i e_i^2) and for the flooring of the quantised weights
 * ((a + 1) 2^-k / sum w).
 * Tie slots take the given ancestor (counted when it differs); non-tie slots
 * keep this run's ancestor, and any difference there is counted.
 * The run stops at an event beyond the E given ones.
 *
 * Outputs (any may be NULL):
 *   scal[5]    = {log Z-hat, final ESS, resamplings, status, factors run}
 *   logz_inc[T] normaliser increment added after factor s (0 where none)
 *   ess_tr[T]  FP64 ESS after factor s
 *   ev[E][8]   per event: {factor s, max mixed |lw' - lw| / max(1, |lw|),
 *              tie slots, adopted tie slots, non-tie differences,
 *              expected tie slots sum_a N * 2 band_a, max band, 0}
 *   dec[3]     = {decisions adopted inside the band, decisions that differ
 *              outside it, decisions inside the band}
 *   mv_out[E][4] with move_steps > 0: per event the move statistics of
 *              gmm_moves (tie decisions, adopted, non-tie differences, max
 *              relative log-alpha difference); g_alpha[E][M][N] the other
 *              run's FP64 log alphas
 *   state_out[n_fields][N], lw_out[N]: particles and log-weights when the run ends */
int or_smc_forced(int32_t model, const double *y, int64_t T, int32_t K, const double *hyper,
                  int64_t N, uint64_t seed, uint32_t inst, double ess_frac, double ess_band,
                  const uint8_t *g_res, const int32_t *g_anc, const float *g_lw, int64_t E,
                  double *scal, double *logz_inc, double *ess_tr, double *ev_out, double *dec,
                  double *state_out, double *lw_out,
                  int32_t move_steps, double move_scale, const double *g_alpha, double *mv_out)
{
    if (N <= 0 || T < 0 || E < 0 || move_steps < 0 || !g_res || (E > 0 && (!g_anc || !g_lw))) return -1;
    if (move_steps > 0 && (model != MODEL_GMM || (E > 0 && !g_alpha))) return -1;
    if (model != MODEL_LGSSM && model != MODEL_GMM) return -2;
    if (model == MODEL_GMM && (K < 1 || K > 8)) return -1;
    int nf = model == MODEL_LGSSM ? 1 : 2 * K;
    double *st = (double *)malloc(sizeof(double) * N * nf);
    double *st2 = (double *)malloc(sizeof(double) * N * nf);
    double *lw = (double *)calloc(N, sizeof(double));
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * N);
    if (!st || !st2 || !lw || !anc) { free(st); free(st2); free(lw); free(anc); return -3; }
    smc_init_state(model, K, hyper, N, seed, inst, st);
    if (dec) dec[0] = dec[1] = dec[2] = 0.0;
    if (logz_inc) for (int64_t s = 0; s < T; ++s) logz_inc[s] = 0.0;

    nsum logz = {0, 0};
    int64_t nres = 0, s_run = 0;
    double ess = (double)N, stat[5];
    int status = 0, stopped = 0;
    for (int64_t s = 0; s < T; ++s) {
        smc_advance(model, K, hyper, y, s, N, seed, inst, st, lw);
        s_run = s + 1;
        or_lse_ess(lw, N, stat);
        if (!(stat[0] > -INFINITY) || isnan(stat[3])) { status = -7; ess = 0.0; break; }
        ess = stat[4];
        if (ess_tr) ess_tr[s] = ess;
        int own = (s < T - 1) && (ess < ess_frac * (double)N);
        int given = (s < T - 1) && g_res[s];
        int in_band = fabs(ess / (double)N - ess_frac) <= ess_band;
        if (dec) {
            if (in_band) dec[2] += 1.0;
            if (in_band && own != given) dec[0] += 1.0;
            if (!in_band && own != given) dec[1] += 1.0;
        }
        if (!given) continue;
        if (nres >= E) { stopped = 1; s_run = s; break; }
        /* this event's normaliser */
        double inc = stat[3] - log((double)N);
        nadd(&logz, inc);
        if (logz_inc) logz_inc[s] = inc;
        int rc = or_forced_event(lw, g_lw + nres * N, g_anc + nres * N, N, seed, (uint32_t)s, inst,
                                 anc, ev_out ? ev_out + nres * 8 : NULL);
        if (rc) { status = rc; break; }
        if (ev_out) ev_out[nres * 8] = (double)s;
        for (int64_t j = 0; j < N; ++j)
            if (anc[j] < 0 || anc[j] >= N) { status = -5; break; }
        if (status) break;
        for (int f = 0; f < nf; ++f)
            for (int64_t j = 0; j < N; ++j) st2[f * N + j] = st[f * N + anc[j]];
        double *tmp = st; st = st2; st2 = tmp;
        if (move_steps > 0)
            gmm_moves(K, hyper, y, s, N, seed, inst, move_steps, move_scale, st, NULL,
                      g_alpha + (size_t)nres * move_steps * N, mv_out ? mv_out + nres * 4 : NULL);
        for (int64_t j = 0; j < N; ++j) lw[j] = 0.0;
        ++nres;
    }
    if (status == 0 && !stopped) {
        if (T > 0) {
            or_lse_ess(lw, N, stat);
            double inc = stat[3] - log((double)N);
            nadd(&logz, inc);
            if (logz_inc) logz_inc[T - 1] = inc;
            ess = stat[4];
        } else {
            ess = (double)N;
        }
    }
    if (scal) {
        scal[0] = status == 0 ? nval(logz) : -INFINITY;
        scal[1] = ess; scal[2] = (double)nres; scal[3] = status; scal[4] = (double)s_run;
    }
    if (state_out) memcpy(state_out, st, sizeof(double) * N * nf);
    if (lw_out) memcpy(lw_out, lw, sizeof(double) * N);
    free(st); free(st2); free(lw); free(anc);
    return status;
}

/* Per-particle GMM initial state (tests of the Dirichlet / Normal prior draws). */
void or_gmm_init(uint64_t seed, uint32_t inst, int32_t K, const double *hyper,
                 int64_t N, double *state /* [2K][N] */)
{
    for (int64_t i = 0; i < N; ++i) {
        double lpi[8], mu[8];
        gmm_init_particle(seed, i, inst, K, hyper, lpi, mu);
        for (int k = 0; k < K; ++k) { state[k * N + i] = lpi[k]; state[(K + k) * N + i] = mu[k]; }
    }
}

/* ------------------------------------------------ learned proposal: data -- */
/* Training pairs are simulated from the model's own prior (Philox tag 4,
 * counter (sample i, block, training step t, 4)):
 *   POLY: block 0 word 0 -> n; blocks 1, 2 -> eight single-precision normals,
 *         c_j = sd z_j; points come in pairs: block 8 + e gives x_{2e}, x_{2e+1}
 *         = 2u - 1 from words 0, 1 and a Box-Muller pair from words 2, 3 for the
 *         observation noise; y = sum_{j<n} c_j x^j + noise_sd * eps.
 *   GMM:  blocks 0, 1 -> Exp(1) draws E_k, pi = E / sum E; blocks 2, 3 -> mu_k =
 *         mu_sd z_k; block 8 + e gives the components of points 2e, 2e+1 from
 *         words 0, 1 (categorical on pi) and their noise from words 2, 3. */
enum { TAG_TRAIN = 4 };
#define SUMM 64

static int categorical(double u, const double *p, int K)
{
    double c = 0.0;
    for (int k = 0; k < K; ++k) { c += p[k]; if (u < c) return k; }
    return K - 1;
}

/* Cholesky solve of the n x n SPD system G beta = m (in place on copies). */
static void chol_solve(int n, const double *G, const double *m, double *beta)
{
    double L[5][5] = {{0}};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = G[i * 5 + j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = (i == j) ? sqrt(s > 1e-300 ? s : 1e-300) : s / L[j][j];
        }
    double z[5];
    for (int i = 0; i < n; ++i) { double s = m[i]; for (int k = 0; k < i; ++k) s -= L[i][k] * z[k]; z[i] = s / L[i][i]; }
    for (int i = n - 1; i >= 0; --i) { double s = z[i]; for (int k = i + 1; k < n; ++k) s -= L[k][i] * beta[k]; beta[i] = s / L[i][i]; }
}

/* POLY summary statistics (64 slots, 42 used):
 *   [0..7]   (1/D) sum x^j y / 10, j = 0..7
 *   [8..21]  (1/D) sum x^k, k = 1..14
 *   [22]     (1/D) sum y^2 / 100
 *   [23..36] least-squares coefficients for n = 2, 3, 4, 5 (n values each) / 10
 *   [37..40] log(1 + (RSS_n - RSS_5) / 2) / 10, RSS_n = D ((1/D) sum y^2 - beta_n . m_n)
 *            clamped at 0: the log-likelihood gap of the n-coefficient fit
 *   [41]     log(D) / 10 */
void or_summary_poly(const double *x, const double *y, int64_t D, double *s)
{
    for (int k = 0; k < SUMM; ++k) s[k] = 0.0;
    if (D <= 0) return;
    double mxy[8] = {0}, gx[15] = {0}, syy = 0.0;
    for (int64_t d = 0; d < D; ++d) {
        double p = 1.0;
        for (int k = 0; k <= 14; ++k) {
            if (k < 8) mxy[k] += p * y[d];
            gx[k] += p;
            p *= x[d];
        }
        syy += y[d] * y[d];
    }
    for (int k = 0; k < 8; ++k) mxy[k] /= (double)D;
    for (int k = 0; k <= 14; ++k) gx[k] /= (double)D;
    syy /= (double)D;
    for (int j = 0; j < 8; ++j) s[j] = mxy[j] / 10.0;
    for (int k = 1; k <= 14; ++k) s[7 + k] = gx[k];
    s[22] = syy / 100.0;
    int o = 23;
    double rss[4];
    for (int n = 2; n <= 5; ++n) {
        double G[25], beta[5];
        for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) G[i * 5 + j] = gx[i + j];
        chol_solve(n, G, mxy, beta);
        double fit = 0.0;
        for (int j = 0; j < n; ++j) { s[o + j] = beta[j] / 10.0; fit += beta[j] * mxy[j]; }
        rss[n - 2] = syy - fit;
        if (rss[n - 2] < 0.0) rss[n - 2] = 0.0;
        o += n;
    }
    for (int n = 2; n <= 5; ++n) {
        double gap = (double)D * (rss[n - 2] - rss[3]) / 2.0;
        if (gap < 0.0) gap = 0.0;
        s[37 + n - 2] = log1p(gap) / 10.0;
    }
    s[41] = log((double)D) / 10.0;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* GMM summary statistics (64 slots, 53 used):
 *   [0..15]  order statistics y_(floor((q + 1/2) D / 16)) / 10, q = 0..15
 *   [16..47] histogram of y on unit bins over [-16, 16) (ends clamped), / D
 *   [48] mean / 10, [49] sd / 10, [50] skewness, [51] excess kurtosis / 10,
 *   [52] log(D) / 10 */
void or_summary_gmm(const double *y, int64_t D, double *s)
{
    for (int k = 0; k < SUMM; ++k) s[k] = 0.0;
    if (D <= 0) return;
    double *v = (double *)malloc(sizeof(double) * D);
    memcpy(v, y, sizeof(double) * D);
    qsort(v, D, sizeof(double), cmp_double);
    for (int q = 0; q < 16; ++q) s[q] = v[(int64_t)floor((q + 0.5) * (double)D / 16.0)] / 10.0;
    free(v);
    double m1 = 0.0;
    for (int64_t d = 0; d < D; ++d) {
        int b = (int)floor(y[d] + 16.0);
        if (b < 0) b = 0;
        if (b > 31) b = 31;
        s[16 + b] += 1.0;
        m1 += y[d];
    }
    for (int b = 0; b < 32; ++b) s[16 + b] /= (double)D;
    m1 /= (double)D;
    double c2 = 0.0, c3 = 0.0, c4 = 0.0;
    for (int64_t d = 0; d < D; ++d) { double r = y[d] - m1; c2 += r * r; c3 += r * r * r; c4 += r * r * r * r; }
    c2 /= (double)D; c3 /= (double)D; c4 /= (double)D;
    double sd = sqrt(c2);
    s[48] = m1 / 10.0;
    s[49] = sd / 10.0;
    s[50] = c2 > 0 ? c3 / (c2 * sd) : 0.0;
    s[51] = c2 > 0 ? (c4 / (c2 * c2) - 3.0) / 10.0 : 0.0;
    s[52] = log((double)D) / 10.0;
}

/* One POLY training pair: theta = (n, c_0..c_4), summaries s[64].
 * hyper = {sd, n_lo, n_hi, noise_sd}. */
void or_sim_poly(uint64_t seed, uint32_t step, int64_t i0, int64_t B, int64_t D, const double *hyper,
                 double *theta, double *summ)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < B; ++b) {
        uint32_t i = (uint32_t)(i0 + b), w[4];
        draw4(seed, i, 0, step, 0, TAG_TRAIN, w);
        int n = (int)or_uniform_discrete(w[0], (int64_t)hyper[1], (int64_t)hyper[2]);
        double z[8];
        draw4(seed, i, 1, step, 0, TAG_TRAIN, w); normals4_single(w, z);
        draw4(seed, i, 2, step, 0, TAG_TRAIN, w); normals4_single(w, z + 4);
        double c[5];
        for (int j = 0; j < 5; ++j) c[j] = hyper[0] * z[j];
        double *x = (double *)malloc(sizeof(double) * D), *y = (double *)malloc(sizeof(double) * D);
        for (int64_t d = 0; d < D; d += 2) {
            draw4(seed, i, (uint32_t)(8 + d / 2), step, 0, TAG_TRAIN, w);
            double e0, e1;
            or_box_muller(or_u01_single(w[2]), or_u01_single(w[3]), &e0, &e1);
            for (int h = 0; h < 2 && d + h < D; ++h) {
                double xv = 2.0 * or_u01_single(w[h]) - 1.0, p = 0.0;
                for (int j = n - 1; j >= 0; --j) p = p * xv + c[j];
                x[d + h] = xv;
                y[d + h] = p + hyper[3] * (h ? e1 : e0);
            }
        }
        theta[b * 6] = n;
        for (int j = 0; j < 5; ++j) theta[b * 6 + 1 + j] = j < n ? c[j] : 0.0;
        or_summary_poly(x, y, D, summ + b * SUMM);
        free(x); free(y);
    }
}

/* One GMM training pair: latents in the ordered unconstrained space
 * u = (mu_(1), log(mu_(k) - mu_(k-1)) for k = 2..K, log pi_(k) - log pi_(K) for
 * k = 1..K-1) (2K - 1 values), summaries s[64].  hyper = {mu_sd, comp_sd}. */
void or_sim_gmm(uint64_t seed, uint32_t step, int64_t i0, int64_t B, int64_t D, int32_t K, const double *hyper,
                double *u, double *summ)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < B; ++b) {
        uint32_t i = (uint32_t)(i0 + b), w[8], v[4];
        draw4(seed, i, 0, step, 0, TAG_TRAIN, w);
        draw4(seed, i, 1, step, 0, TAG_TRAIN, w + 4);
        double E[8], tot = 0.0, pi[8], mu[8], z[8];
        for (int k = 0; k < K; ++k) { E[k] = -log(or_u01_single(w[k])); tot += E[k]; }
        for (int k = 0; k < K; ++k) pi[k] = E[k] / tot;
        draw4(seed, i, 2, step, 0, TAG_TRAIN, v); normals4_single(v, z);
        draw4(seed, i, 3, step, 0, TAG_TRAIN, v); normals4_single(v, z + 4);
        for (int k = 0; k < K; ++k) mu[k] = hyper[0] * z[k];
        double *y = (double *)malloc(sizeof(double) * D);
        for (int64_t d = 0; d < D; d += 2) {
            draw4(seed, i, (uint32_t)(8 + d / 2), step, 0, TAG_TRAIN, v);
            double e0, e1;
            or_box_muller(or_u01_single(v[2]), or_u01_single(v[3]), &e0, &e1);
            for (int h = 0; h < 2 && d + h < D; ++h) {
                int k = categorical(or_u01_single(v[h]), pi, K);
                y[d + h] = mu[k] + hyper[1] * (h ? e1 : e0);
            }
        }
        /* sort components by mean (insertion sort, ties keep index order) */
        int ord[8] = {0, 1, 2, 3, 4, 5, 6, 7};
        for (int a = 1; a < K; ++a)
            for (int c = a; c > 0 && mu[ord[c]] < mu[ord[c - 1]]; --c) { int t = ord[c]; ord[c] = ord[c - 1]; ord[c - 1] = t; }
        double *ub = u + b * (2 * K - 1);
        ub[0] = mu[ord[0]];
        for (int k = 1; k < K; ++k) ub[k] = log(mu[ord[k]] - mu[ord[k - 1]]);
        for (int k = 0; k < K - 1; ++k) ub[K + k] = log(pi[ord[k]]) - log(pi[ord[K - 1]]);
        or_summary_gmm(y, D, summ + b * SUMM);
        free(y);
    }
}

/* -------------------------------------------- learned proposal: weights -- */
static double log_normal(double v, double m, double lsd)
{
    double r = (v - m) * exp(-lsd);
    return -0.5 * r * r - lsd - 0.5 * log(2.0 * M_PI);
}

static double lse(const double *v, int n)
{
    double m = -INFINITY;
    for (int k = 0; k < n; ++k) if (v[k] > m) m = v[k];
    if (!(m > -INFINITY)) return -INFINITY;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += exp(v[k] - m);
    return m + log(s);
}

/* log q(n, c) of the POLY proposal: params = {lognl[4] (log-softmax of the degree
 * logits), logmix[8] (log-softmax of the mixture logits), mean[4][8][5], lsd[4][8][5]}. */
double or_poly_logq(const double *params, int n, const double *c)
{
    const double *lnl = params, *lmix = params + 4, *mean = params + 12, *lsd = params + 12 + 160;
    double t[8];
    for (int m = 0; m < 8; ++m) {
        t[m] = lmix[m];
        for (int j = 0; j < n; ++j)
            t[m] += log_normal(c[j], mean[((n - 2) * 8 + m) * 5 + j], lsd[((n - 2) * 8 + m) * 5 + j]);
    }
    return lnl[n - 2] + lse(t, 8);
}

/* Importance weights of the POLY model under the proposal (PROPOSAL stream:
 * block 0 words 0, 1 -> degree and component; blocks 1, 2 -> normals; c_j =
 * mean + exp(lsd) z_j in single precision as drawn, then everything in FP64):
 * lw = log p(n, c) + log L(c) - log q(n, c).  hyper = {sd, n_lo, n_hi}. */
void or_propose_poly(uint64_t seed, const double *params, const double *x, const double *y, int64_t D,
                     const double *hyper, int64_t m, const int64_t *idx, double *lw, double *draw /* [m][6] */)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < m; ++r) {
        uint32_t i = (uint32_t)idx[r], w[4];
        draw4(seed, i, 0, 0, 0, TAG_PROPOSAL, w);
        double pn[4], pm[8];
        for (int k = 0; k < 4; ++k) pn[k] = exp(params[k]);
        for (int k = 0; k < 8; ++k) pm[k] = exp(params[4 + k]);
        int n = 2 + categorical(or_u01_single(w[0]), pn, 4);
        int comp = categorical(or_u01_single(w[1]), pm, 8);
        double z[8], c[5];
        draw4(seed, i, 1, 0, 0, TAG_PROPOSAL, w); normals4_single(w, z);
        draw4(seed, i, 2, 0, 0, TAG_PROPOSAL, w); normals4_single(w, z + 4);
        for (int j = 0; j < 5; ++j) {
            const double *mean = params + 12, *lsd = params + 12 + 160;
            int o = ((n - 2) * 8 + comp) * 5 + j;
            c[j] = j < n ? mean[o] + exp(lsd[o]) * z[j] : 0.0;
        }
        double lp = -log(4.0);
        for (int j = 0; j < n; ++j) lp += log_normal(c[j], 0.0, log(hyper[0]));
        lw[r] = lp + or_poly_loglik(n, c, x, y, D) - or_poly_logq(params, n, c);
        draw[r * 6] = n;
        for (int j = 0; j < 5; ++j) draw[r * 6 + 1 + j] = c[j];
    }
}

/* GMM (K components) proposal over the ordered unconstrained latents u (2K - 1):
 * params = {logmix[8], mean[8][2K-1], lsd[8][2K-1]}. */
double or_gmm_logq(const double *params, int32_t K, const double *u)
{
    const int d = 2 * K - 1;
    const double *lmix = params, *mean = params + 8, *lsd = params + 8 + 8 * d;
    double t[8];
    for (int m = 0; m < 8; ++m) {
        t[m] = lmix[m];
        for (int i = 0; i < d; ++i) t[m] += log_normal(u[i], mean[m * d + i], lsd[m * d + i]);
    }
    return lse(t, 8);
}

/* Map u to (log pi, mu) and return the prior density of u:
 * log p(u) = log (K-1)! [Dirichlet(1)] + log K! [ordering] + sum_k log N(mu_k; 0, mu_sd)
 *          + sum_{k>=2} u_k [d mu / d gaps] + sum_k log pi_k [softmax Jacobian]. */
double or_gmm_unpack(const double *u, int32_t K, double mu_sd, double *lpi, double *mu)
{
    mu[0] = u[0];
    for (int k = 1; k < K; ++k) mu[k] = mu[k - 1] + exp(u[k]);
    double lg[8];
    for (int k = 0; k < K - 1; ++k) lg[k] = u[K + k];
    lg[K - 1] = 0.0;
    double z = lse(lg, K);
    double lp = lgamma((double)K) + lgamma((double)K + 1.0);
    for (int k = 0; k < K; ++k) {
        lpi[k] = lg[k] - z;
        lp += log_normal(mu[k], 0.0, log(mu_sd)) + lpi[k];
        if (k >= 1) lp += u[k];
    }
    return lp;
}

/* Importance weights of the GMM model under the proposal (PROPOSAL stream:
 * block 0 word 0 -> component; blocks 1..4 -> sixteen normals, z_k for u_k):
 * lw = log p(u) + log L(u) - log q(u).  hyper = {mu_sd, comp_sd}. */
void or_propose_gmm(uint64_t seed, const double *params, int32_t K, const double *y, int64_t D,
                    const double *hyper, int64_t m, const int64_t *idx, double *lw, double *draw /* [m][2K-1] */)
{
    const int dim = 2 * K - 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < m; ++r) {
        uint32_t i = (uint32_t)idx[r], w[4];
        draw4(seed, i, 0, 0, 0, TAG_PROPOSAL, w);
        double pm[8], z[16], u[15], lpi[8], mu[8];
        for (int k = 0; k < 8; ++k) pm[k] = exp(params[k]);
        int comp = categorical(or_u01_single(w[0]), pm, 8);
        for (int b = 0; b < 4; ++b) { draw4(seed, i, (uint32_t)(1 + b), 0, 0, TAG_PROPOSAL, w); normals4_single(w, z + 4 * b); }
        for (int k = 0; k < dim; ++k) u[k] = params[8 + comp * dim + k] + exp(params[8 + 8 * dim + comp * dim + k]) * z[k];
        double lp = or_gmm_unpack(u, K, hyper[0], lpi, mu);
        double ll = 0.0;
        for (int64_t d = 0; d < D; ++d) ll += or_gmm_logfactor(K, lpi, mu, hyper[1], y[d]);
        lw[r] = lp + ll - or_gmm_logq(params, K, u);
        for (int k = 0; k < dim; ++k) draw[r * dim + k] = u[k];
    }
}

/* Prior-proposal importance weights of the GMM model (PRIOR stream, the same
 * draws as the SMC initial particles): lw = log L(pi, mu). */
void or_gmm_prior_lw(uint64_t seed, int32_t K, const double *hyper, const double *y, int64_t D, int64_t m,
                     const int64_t *idx, double *lw)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < m; ++r) {
        double lpi[8], mu[8];
        gmm_init_particle(seed, idx[r], 0, K, hyper, lpi, mu);
        double ll = 0.0;
        for (int64_t d = 0; d < D; ++d) ll += or_gmm_logfactor(K, lpi, mu, hyper[1], y[d]);
        lw[r] = ll;
    }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Host threads for the particle loops of later calls (n < 1: all available). */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n < 1) n = omp_get_num_procs();
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}
