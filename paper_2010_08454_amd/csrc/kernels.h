// kernels.h -- launch entry points shared between the C ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppl {

struct IsArgs {
    int model;
    const void *x, *y;
    int64_t D;
    int dim;
    double hyper[8];
    int64_t N;
    uint64_t seed;
    const void *q_params;   // proposal parameters (BLR: float32 mean + Cholesky; POLY / GMM: FP64 mixture) or null
    void *lw_out, *lat_out;
    double *scalars;        // [8], device
    double *summaries;      // device or null
    double *part;           // workspace: per-block partial records
};

size_t is_partial_bytes(int model, int dim, int64_t N);
int run_importance(const IsArgs &a, hipStream_t st);

// Mixture-proposal importance sampling (POLY with q, GMM with or without q).
size_t prop_partial_bytes(int model, int64_t N);
int run_importance_q(const IsArgs &a, hipStream_t st);

// BLR with the likelihood from sufficient statistics (PPL_MODEL_BLR_STATS):
// workspace bytes after the 256-byte scalar slot, and the launcher (a.part is
// that workspace).
size_t blr_stats_ws_bytes(int dim, int64_t N, int64_t D);
int run_importance_blr_stats(const IsArgs &a, hipStream_t st);

// Normaliser of a device log-weight vector (see ppl_lse_ess).
size_t lse_ws_bytes(int64_t n);
int run_lse(const void *lw, bool f64, int64_t n, double *out5, void *ws, hipStream_t st);

// Integer-rule systematic resampling (see ppl_resample).
size_t resample_ws_bytes(int64_t n);
int run_resample(const void *lw, bool f64, int64_t n, uint64_t seed, uint32_t step, uint32_t inst,
                 int32_t *anc, void *ws, hipStream_t st);
// Resampling fused with the gather of nf 32-bit state fields (see ppl_resample_gather).
int run_resample_gather(const void *lw, bool f64, int64_t n, uint64_t seed, uint32_t step, uint32_t inst, int nf,
                        const void *state_in, void *state_out, int32_t *anc, void *ws, hipStream_t st);

// Enumeration of every path of a hidden Markov model (see ppl_enumerate).
struct EnumArgs {
    int K, T;
    const double *y;            // [T] device
    double sigma;
    const double *pi0, *A, *mu; // host: [K], [K][K], [K]
    double *scalars;            // [4] device
    double *marginals;          // [T][K] device or null
    int32_t *map;               // [T] device or null
    void *ws;
};
size_t enum_ws_bytes(int K, int T);
int run_enumerate_hmm(const EnumArgs &a, hipStream_t st);

int run_philox(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t *out, hipStream_t st);

}  // namespace ppl
