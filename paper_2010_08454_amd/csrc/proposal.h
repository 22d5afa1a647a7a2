// proposal.h -- learned proposal: simulated training pairs, data summaries,
// network training and the decoded mixture proposal (launchers shared by the
// C ABI layer).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.h"

namespace ppl {

constexpr int kSummaryDim = 64;      // summary statistics per dataset (network input)
constexpr int kThetaStride = 16;     // FP64 latent slots per training pair
constexpr int kHeadComps = 8;        // mixture components of the proposal
constexpr int kPolyQParams = 12 + 2 * 160;   // lognl[4], logmix[8], mean[4][8][5], lsd[4][8][5]
inline int gmm_q_params(int K) { return 8 + 16 * (2 * K - 1); }
constexpr int kGmmSummaryMaxD = 8192;        // observed-data limit of the mixture summaries (32 KB of LDS)
constexpr int kGmmTrainMaxD = 4096;          // per simulated dataset (one per workgroup, 32 KB of LDS)

// Simulation hyper-parameters.  POLY: {sd, n_lo, n_hi, noise_sd};
// GMM: {mu_sd, comp_sd}, with K components.
struct SimSpec {
    int model;
    int K;
    int64_t D;
    double hyper[4];
};

// Simulate B training pairs of training step `*step` (Philox tag 4, counter
// (pair, block, step, 4)) and write their summaries as BF16 rows x_row[B][64]
// and columns x_col[64][B], the latents theta[B][16] (FP64) and, if s64 is not
// null, the FP64 summaries s64[B][64].
int launch_simulate(const SimSpec &sp, int B, uint64_t seed, const int64_t *step, uint16_t *x_row, uint16_t *x_col,
                    double *theta, double *s64, hipStream_t st);

// Summaries of one observed dataset into row 0 of x_row[64][64] (rows 1..63
// cleared) and, if s64 is not null, the FP64 values s64[64].
int launch_observed_summary(int model, const void *x, const void *y, int64_t D, uint16_t *x_row, double *s64,
                            hipStream_t st);

// Training-step buffers (device), all allocated from one workspace.
struct TrainBufs {
    int B;
    uint16_t *x_row, *x_col;            // [B][64], [64][B]
    double *theta;                      // [B][16]
    uint16_t *h1_row, *h1_col, *h2_row, *h2_col;   // [B][256], [256][B]
    float *o_col;                       // [256][B]
    uint16_t *do_row, *do_col, *dh2_row, *dh2_col, *dh1_col;
    float *part[3];                     // split-R partials of dW_l
    int nchunks[3], chunk[3];
    float *bgrad;                       // [3][256]
    double *lossp;                      // [B / 32] per-workgroup loss sums
    int64_t *local;                     // [0]: steps taken in this call, [1]: a fixed step index
    float *coef;                        // [3] Adam constants of the step being taken: 1 - b1^t, 1 - b2^t, lr
};

size_t train_ws_bytes(int B);
TrainBufs train_bufs(void *ws, int B);

struct AdamSpec {
    float lr, b1, b2, eps;
    double decay_steps;      // > 0: half-cosine decay of lr over this many steps
    double final_frac;       // lr multiplier reached at the end of the decay
};

// Per-step bookkeeping, run once by one wave after the loss partials are
// written and before the Adam update: loss_trace[local] = mean loss,
// local += 1 and, if step is not null, the Adam constants of step
// t = step + 1 into coef, then step += 1.
struct AdvanceJob {
    int64_t *step, *local;
    const double *lossp;
    int nparts;
    double inv_b;
    double *loss_trace;
    AdamSpec ad;
    float *coef;
};
AdvanceJob advance_job(int64_t *step, const TrainBufs &b, const AdamSpec &ad, double *loss_trace);

// Forward pass of a batch whose summaries are already in bufs.x_row/x_col.
int launch_forward(const MlpView &w, const TrainBufs &b, bool keep_cols, hipStream_t st);
// Loss head and backward pass (gradients left in the split partials and bgrad).
int launch_head_backward(int model, int K, const MlpView &w, const TrainBufs &b, hipStream_t st);
// The same in fewer launches: forward, head and input gradients fused per 32
// pairs (bitwise the values of launch_forward + launch_head_backward), then
// the weight-gradient products, bias sums and the step's bookkeeping (adv).
int launch_fused_pass(int model, int K, const MlpView &w, const TrainBufs &b, const AdvanceJob &adv, hipStream_t st);
// grad != null: write the summed gradient [count] and stop; else Adam update
// with the constants the step's bookkeeping left in b.coef.
int launch_update(const MlpView &w, const TrainBufs &b, const AdamSpec &ad, float *grad, hipStream_t st);
// The step's bookkeeping as a launch of its own (after launch_head_backward).
int launch_advance(const AdvanceJob &adv, hipStream_t st);
// launch_update (Adam, grad null) and launch_simulate of the next batch into
// b.x_row, b.x_col, b.theta, in one launch; step must already be advanced.
int launch_update_simulate(const MlpView &w, const TrainBufs &b, const AdamSpec &ad, const SimSpec &sp, int B,
                           uint64_t seed, const int64_t *step, hipStream_t st);
int launch_set_i64(int64_t *p, int64_t v, hipStream_t st);
int launch_init_weights(void *weights, uint64_t seed, hipStream_t st);

// Decode the network output column 0 of o_col[256][ld] into FP64 proposal
// parameters (kPolyQParams or gmm_q_params(K) values); log_widen is added to
// every used log-scale.
int launch_decode(int model, int K, const float *o_col, int ld, double log_widen, double *q, hipStream_t st);

}  // namespace ppl
