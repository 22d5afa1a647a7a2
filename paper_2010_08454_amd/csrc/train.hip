// train.hip -- training of the proposal network: mixture-density loss head,
// backward pass, Adam, weight initialisation and the decoded proposal.
//
// The network (64 -> 256 -> 256 -> 256, ReLU after the first two layers, BF16
// MFMA products with FP32 accumulation) maps the summaries s(y) of a dataset
// to the parameters of an 8-component diagonal Gaussian mixture q(theta | y)
// over the model's latents; the loss is the mean of -log q(theta_i | y_i)
// over pairs (theta_i, y_i) simulated from the model's prior.  BF16 is stored
// at the network inputs, the weights, the hidden activations and the
// back-propagated gradients; biases, FP32 master weights and Adam moments
// stay FP32.
//
// Output head (256 network outputs o):
//   POLY: o[0:4] degree logits (n = 2..5), o[4:12] mixture logits shared by
//         all degrees; for degree n a block at 12 + 8 (n - 2)(n + 1) holding
//         8n means (10 o) then 8n log-scales (5 tanh(o / 5)), component-major.
//   GMM (K components, d = 2K - 1 ordered unconstrained latents): o[0:8]
//         mixture logits, o[8 : 8 + 8d] means (5 o), then 8d log-scales.
#include "adam.h"
#include "device.h"
#include "host.h"
#include "proposal.h"
#include "timing.h"

namespace ppl {

constexpr float kHalfLog2Pi = 0.91893853320467274f;
constexpr uint32_t kTagInit = 5;
constexpr int kLdsRow = 258;          // BF16 per LDS row of the head (odd word stride)

__host__ __device__ constexpr int poly_head_off(int n) { return 12 + 8 * (n - 2) * (n + 1); }

// ---------------------------------------------------------------- head --
// Eight lanes per training pair, lane m owning mixture component m; 32 pairs
// per 256-thread workgroup.  The component sums (log-softmax, log-sum-exp over
// components) are butterflies within the 8-lane group.  The gradient of the
// loss w.r.t. the outputs, divided by the batch size, is rounded to BF16 and
// staged in LDS, so both the row-major and the column-major copies are
// written with contiguous stores.
constexpr int kHeadPairs = 32;

__device__ __forceinline__ float group8_max(float v) {
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float group8_sum(float v) {
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The loss of one training pair and its gradient w.r.t. the network outputs:
// lane m (0..7) of the pair's 8-lane group owns mixture component m; output k
// is o[k os]; the BF16 gradient (divided by the batch size) goes to g[k],
// whose unused entries the caller has zeroed.  Returns the pair's loss on
// lane 0 and 0 elsewhere.
template <int MODEL>
__device__ __forceinline__ float head_pair(const float *o, int os, const double *th, int K, float inv_b, uint16_t *g,
                                           int m) {
    auto O = [&](int k) { return o[(size_t)k * os]; };
    float loss;
    // mixture weights: lane m's log-softmax entry
    const int mix0 = MODEL == PPL_MODEL_POLY ? 4 : 0;
    const float zm = O(mix0 + m);
    const float mm = group8_max(zm);
    const float lse_m = mm + logf(group8_sum(expf(zm - mm)));
    const float lmix = zm - lse_m;
    float t = lmix;
    if constexpr (MODEL == PPL_MODEL_POLY) {
        const int n = min(max((int)th[0], 2), 5);
        const int off = poly_head_off(n);
        // per coefficient: th5 = tanh(z / 5), iv = exp(-5 th5) (the inverse
        // scale), dv = theta - mu; kept for the gradient below
        float th5v[5], ivv[5], dvv[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            th5v[j] = ivv[j] = dvv[j] = 0.0f;
            if (j < n) {
                const float mu = 10.0f * O(off + m * n + j);
                const float th5 = tanhf(O(off + 8 * n + m * n + j) * 0.2f);
                const float lsd = 5.0f * th5;
                const float iv = expf(-lsd);
                const float dv = (float)th[1 + j] - mu;
                const float r = dv * iv;
                t += -0.5f * r * r - lsd - kHalfLog2Pi;
                th5v[j] = th5;
                ivv[j] = iv;
                dvv[j] = dv;
            }
        }
        const float tm = group8_max(t);
        const float L = tm + logf(group8_sum(expf(t - tm)));
        const float resp = expf(t - L);
        // degree term: lanes 0..3 own degree n = 2 + m
        float zn[4], mx = -INFINITY;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            zn[k] = O(k);
            mx = fmaxf(mx, zn[k]);
        }
        float se = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) se += expf(zn[k] - mx);
        const float lse_n = mx + logf(se);
        float zsel = zn[0];
#pragma unroll
        for (int k = 1; k < 4; ++k) zsel = (k == n - 2) ? zn[k] : zsel;
        loss = m == 0 ? -(zsel - lse_n) - L : 0.0f;
        if (m < 4) {
            float zk = zn[0];
#pragma unroll
            for (int k = 1; k < 4; ++k) zk = (k == m) ? zn[k] : zk;
            g[m] = f32_to_bf16((expf(zk - lse_n) - (m == n - 2 ? 1.0f : 0.0f)) * inv_b);
        }
        g[4 + m] = f32_to_bf16((expf(lmix) - resp) * inv_b);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (j < n) {
                const int km = off + m * n + j, ks = off + 8 * n + m * n + j;
                const float th5 = th5v[j], iv = ivv[j], dv = dvv[j];
                const float r = dv * iv;
                g[km] = f32_to_bf16(-resp * dv * iv * iv * 10.0f * inv_b);
                g[ks] = f32_to_bf16(-resp * (r * r - 1.0f) * (1.0f - th5 * th5) * inv_b);
            }
        }
    } else {
        const int d = 2 * K - 1;
        for (int j = 0; j < d; ++j) {
            const float mu = 5.0f * O(8 + m * d + j);
            const float lsd = 5.0f * tanhf(O(8 + 8 * d + m * d + j) * 0.2f);
            const float r = ((float)th[j] - mu) * expf(-lsd);
            t += -0.5f * r * r - lsd - kHalfLog2Pi;
        }
        const float tm = group8_max(t);
        const float L = tm + logf(group8_sum(expf(t - tm)));
        const float resp = expf(t - L);
        loss = m == 0 ? -L : 0.0f;
        g[m] = f32_to_bf16((expf(lmix) - resp) * inv_b);
        for (int j = 0; j < d; ++j) {
            const int km = 8 + m * d + j, ks = 8 + 8 * d + m * d + j;
            const float mu = 5.0f * O(km);
            const float th5 = tanhf(O(ks) * 0.2f);
            const float iv = expf(-5.0f * th5);
            const float dv = (float)th[j] - mu;
            const float r = dv * iv;
            g[km] = f32_to_bf16(-resp * dv * iv * iv * 5.0f * inv_b);
            g[ks] = f32_to_bf16(-resp * (r * r - 1.0f) * (1.0f - th5 * th5) * inv_b);
        }
    }
    return loss;
}

template <int MODEL>
__global__ __launch_bounds__(256) void head_kernel(const float *__restrict__ o_col, int B,
                                                   const double *__restrict__ theta, int K, float inv_b,
                                                   uint16_t *__restrict__ do_row, uint16_t *__restrict__ do_col,
                                                   double *__restrict__ lossp) {
    __shared__ uint32_t lds32[kHeadPairs * kLdsRow / 2];
    __shared__ double red[4];
    uint16_t *lds = (uint16_t *)lds32;
    const int tid = threadIdx.x, m = tid & 7, sl = tid >> 3;
    const int b0 = blockIdx.x * kHeadPairs, b = b0 + sl;
    for (int k = tid; k < kHeadPairs * kLdsRow / 2; k += 256) lds32[k] = 0u;
    __syncthreads();
    const float loss = head_pair<MODEL>(o_col + b, B, theta + (size_t)b * kThetaStride, K, inv_b,
                                        lds + sl * kLdsRow, m);
    const double ls = wave_sum((double)loss);
    if ((tid & 63) == 0) red[tid >> 6] = ls;
    __syncthreads();
    if (tid == 0) lossp[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    for (int e = tid; e < kHeadPairs * kMlpOut; e += 256) {
        const int k = e / kHeadPairs, q = e % kHeadPairs;
        do_col[(size_t)k * B + b0 + q] = lds[q * kLdsRow + k];
    }
    for (int e = tid; e < kHeadPairs * kMlpOut; e += 256) {
        const int q = e / kMlpOut, k = e % kMlpOut;
        do_row[(size_t)(b0 + q) * kMlpOut + k] = lds[q * kLdsRow + k];
    }
}

// ------------------------------------------------- fused training pass --
// Forward pass, loss head and the input-gradient half of the backward pass for
// 32 training pairs per 256-thread workgroup, in one launch: the hidden
// activations, the network outputs and the output gradients stay in LDS
// between layers (BF16 rows padded to 264 entries, so every 8-entry fragment
// is one aligned 16-byte LDS load).  Each product is C[32][256] = A[32][K]
// B[256][K]^T on v_mfma_f32_16x16x32_bf16, wave w computing columns 64 w ..
// 64 w + 63; fragments and accumulation order over K are those of
// gemm_nt_kernel, and the epilogues round at the same points, so every stored
// value equals the separate launches' bit for bit.  The column-major copies
// the weight gradients and bias sums read (h1, h2, dO, dH2, dH1) and the FP32
// outputs go to global memory.
constexpr int kFuseRows = 32;
constexpr int kFusePad = 264;           // BF16 per LDS row
constexpr int kFuseOPad = 260;          // FP32 per LDS row of the outputs

typedef __bf16 fbf16x8_t __attribute__((ext_vector_type(8)));
typedef float ffloatx4_t __attribute__((ext_vector_type(4)));

// A product's weight fragments for this wave: fb[s][j] holds B rows
// 64 wave + 16 j + lane % 16, K entries 32 s + 8 (lane / 16) .. + 7, read from
// the fragment-order copy of the weights (frag_index: each load instruction
// reads 1 KB of consecutive bytes; from the [out][in] or [in][out] layout a
// wave's load touched 16 rows, 64 bytes of each).  They are loaded one product
// ahead (while the previous product's epilogue and the workgroup barrier run),
// so a product waits for global memory at most once.
typedef fbf16x8_t FuseFrags[8][4];

template <int KD>
__device__ __forceinline__ void fuse_load_w(const uint16_t *Bw, FuseFrags &fb) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
#pragma unroll
    for (int s = 0; s < KD / 32; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            fb[s][j] = *(const fbf16x8_t *)(Bw + frag_index(64 * wave + 16 * j + fr, 32 * s + fk, KD));
    __builtin_amdgcn_sched_barrier(0);       // keep the scheduler from sinking the loads into the MFMA loop
}

// acc[i][j][q] = C[16 i + 4 (lane / 16) + q][64 wave + 16 j + lane % 16] of
// C[32][256] = A[32][KD] B[256][KD]^T, B's fragments in fb.
template <int KD>
__device__ __forceinline__ void fuse_mma(const uint16_t *A, int lda, const FuseFrags &fb, ffloatx4_t (&acc)[2][4]) {
    const int lane = threadIdx.x & 63;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = ffloatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KD / 32; ++s) {
        fbf16x8_t fa[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) fa[i] = *(const fbf16x8_t *)(A + (size_t)(16 * i + fr) * lda + 32 * s + fk);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[s][j], acc[i][j], 0, 0, 0);
    }
}

// Hidden-layer epilogue: relu(acc + bias) in BF16 to LDS rows and to the
// column-major global copy [256][B] (columns b0 .. b0 + 31).
__device__ __forceinline__ void fuse_store_hidden(const ffloatx4_t (&acc)[2][4], const float (&bias)[4], uint16_t *lds,
                                                  uint16_t *col, int B, int b0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fr = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = 64 * wave + 16 * j + fr, mb = 16 * i + rq;
            const float bn = bias[j];
            uint16_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                h[q] = f32_to_bf16(fmaxf(acc[i][j][q] + bn, 0.0f));
                lds[(mb + q) * kFusePad + n] = h[q];
            }
            *(uint2 *)(col + (size_t)n * B + b0 + mb) =
                make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
        }
}

// Input-gradient epilogue: acc masked by the ReLU derivative (nonzero BF16
// activation in `mask`), in BF16 to LDS rows (if lds) and the column-major copy.
__device__ __forceinline__ void fuse_store_masked(const ffloatx4_t (&acc)[2][4], const uint16_t *mask, uint16_t *lds,
                                                  uint16_t *col, int B, int b0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fr = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = 64 * wave + 16 * j + fr, mb = 16 * i + rq;
            uint16_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float t = (mask[(mb + q) * kFusePad + n] & 0x7FFFu) ? acc[i][j][q] : 0.0f;
                h[q] = f32_to_bf16(t);
                if (lds) lds[(mb + q) * kFusePad + n] = h[q];
            }
            *(uint2 *)(col + (size_t)n * B + b0 + mb) =
                make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
        }
}

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations (lgkmcnt 0) but leaves its global stores and the
// prefetched weight loads in flight (a full __syncthreads would wait for
// them at every layer).  Nothing the fused pass stores to global memory is
// read back by another wave of the workgroup.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);      // vmcnt and expcnt: no wait; lgkmcnt: 0
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int MODEL>
__global__ __launch_bounds__(256) void fused_pass_kernel(MlpView w, TrainBufs b, int K, float inv_b) {
    __shared__ __align__(16) uint16_t sH1[kFuseRows * kFusePad];
    __shared__ __align__(16) uint16_t sH2[kFuseRows * kFusePad];
    __shared__ __align__(16) uint16_t sG[kFuseRows * kFusePad];     // dO
    __shared__ __align__(16) uint16_t sD2[kFuseRows * kFusePad];    // dH2
    __shared__ __align__(16) float sO[kFuseRows * kFuseOPad];
    __shared__ double sTh[kFuseRows * kThetaStride];
    __shared__ double red[4];
    const int B = b.B, b0 = blockIdx.x * kFuseRows, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // Global reads that epilogues and the head need are issued first: vector
    // memory loads and stores complete in order, so a load issued after the
    // next product's weight prefetch would wait for that prefetch too.
    float bias_r[3][4];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int j = 0; j < 4; ++j) bias_r[l][j] = w.master[MlpParams::b_off(l) + 64 * wave + 16 * j + (lane & 15)];
    ffloatx4_t acc[2][4];
    FuseFrags fb;
    // layer 1: H1 = relu(X W1^T + b1)
    fuse_load_w<kMlpIn>(w.wtf + MlpParams::bf16_w_off(0), fb);
    for (int e = tid; e < kFuseRows * kThetaStride; e += 256) sTh[e] = b.theta[(size_t)b0 * kThetaStride + e];
    fuse_mma<kMlpIn>(b.x_row + (size_t)b0 * kMlpIn, kMlpIn, fb, acc);
    fuse_load_w<kMlpHid>(w.wtf + MlpParams::bf16_w_off(1), fb);
    fuse_store_hidden(acc, bias_r[0], sH1, b.h1_col, B, b0);
    for (int k = tid; k < kFuseRows * kFusePad / 2; k += 256) ((uint32_t *)sG)[k] = 0u;
    lds_barrier();
    // layer 2: H2 = relu(H1 W2^T + b2)
    fuse_mma<kMlpHid>(sH1, kFusePad, fb, acc);
    fuse_load_w<kMlpHid>(w.wtf + MlpParams::bf16_w_off(2), fb);
    fuse_store_hidden(acc, bias_r[1], sH2, b.h2_col, B, b0);
    lds_barrier();
    // layer 3: O = H2 W3^T + b3 (FP32)
    fuse_mma<kMlpHid>(sH2, kFusePad, fb, acc);
    fuse_load_w<kMlpOut>(w.wf + MlpParams::bf16_w_off(2), fb);
    {
        const int fr = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = 64 * wave + 16 * j + fr, mb = 16 * i + rq;
                const float bn = bias_r[2][j];
                float v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    v[q] = acc[i][j][q] + bn;
                    sO[(mb + q) * kFuseOPad + n] = v[q];
                }
                *(float4 *)(b.o_col + (size_t)n * B + b0 + mb) = make_float4(v[0], v[1], v[2], v[3]);
            }
    }
    lds_barrier();
    // loss head: pair tid / 8, component tid % 8; gradient rows into sG
    {
        const int m = tid & 7, sl = tid >> 3;
        const float loss = head_pair<MODEL>(sO + sl * kFuseOPad, 1, sTh + sl * kThetaStride, K, inv_b,
                                            sG + sl * kFusePad, m);
        const double ls = wave_sum((double)loss);
        if (lane == 0) red[wave] = ls;
    }
    lds_barrier();
    if (tid == 0) b.lossp[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    // dO to the column-major copy: four consecutive pairs of one output per
    // 8-byte store, all LDS reads of a thread issued together
#pragma unroll
    for (int it = 0; it < kFuseRows * kMlpOut / (4 * 256); ++it) {
        const int e = tid + 256 * it;
        const int k = e / (kFuseRows / 4), q = (e % (kFuseRows / 4)) * 4;
        const uint32_t lo = (uint32_t)sG[q * kFusePad + k] | ((uint32_t)sG[(q + 1) * kFusePad + k] << 16);
        const uint32_t hi = (uint32_t)sG[(q + 2) * kFusePad + k] | ((uint32_t)sG[(q + 3) * kFusePad + k] << 16);
        *(uint2 *)(b.do_col + (size_t)k * B + b0 + q) = make_uint2(lo, hi);
    }
    // layer 3 input gradient: dH2 = (dO W3) * [H2 > 0]
    fuse_mma<kMlpOut>(sG, kFusePad, fb, acc);
    fuse_load_w<kMlpHid>(w.wf + MlpParams::bf16_w_off(1), fb);
    fuse_store_masked(acc, sH2, sD2, b.dh2_col, B, b0);
    lds_barrier();
    // layer 2 input gradient: dH1 = (dH2 W2) * [H1 > 0]
    fuse_mma<kMlpHid>(sD2, kFusePad, fb, acc);
    fuse_store_masked(acc, sH1, nullptr, b.dh1_col, B, b0);
}

// ------------------------------------------------------ bias gradients --
// bgrad[l][o] = sum over the batch of the BF16 gradient column o of layer l
// (FP32, a fixed order: 256 strided lane sums, then a tree).
__device__ __forceinline__ void bias_grad_unit(const uint16_t *__restrict__ g1, const uint16_t *__restrict__ g2,
                                               const uint16_t *__restrict__ g3, int B, float *__restrict__ bgrad,
                                               int unit) {
    __shared__ float red[4];
    const int l = unit >> 8, o = unit & 255;
    const uint16_t *g = (l == 0 ? g1 : (l == 1 ? g2 : g3)) + (size_t)o * B;
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) s += bf16_to_f32(g[b]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) bgrad[unit] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void bias_grad_kernel(const uint16_t *__restrict__ g1, const uint16_t *__restrict__ g2,
                                                        const uint16_t *__restrict__ g3, int B,
                                                        float *__restrict__ bgrad) {
    bias_grad_unit(g1, g2, g3, B, bgrad, blockIdx.x);
}

// The three weight-gradient products (split over R-chunks) and the bias sums
// in one launch: workgroups [first_k, first_k + tx ty nz) take product k's
// tiles (x fastest, then y, then the chunk), the rest one bias each.  Every
// tile and bias is computed as by the separate launches, so the bits match.
struct WgradJob {
    const uint16_t *A, *B;
    float *partial;
    int M, N, R, lda, ldb, chunk, tx, ty, first;
};
struct WgradGroup {
    WgradJob job[3];
    int gemm_blocks;
    const uint16_t *g1, *g2, *g3;
    int B;
    float *bgrad;
    AdvanceJob adv;
};

// The step's bookkeeping (one wave): the mean loss from the per-workgroup
// partials, the call's step counter and, when the weights' step count is
// given, the Adam constants of step t = completed steps + 1 (bias
// corrections, the learning rate optionally on a half-cosine schedule of the
// completed steps) computed once for every parameter, then the count.
__device__ void advance_unit(const AdvanceJob &a) {
    double s = 0.0;
    for (int k = threadIdx.x & 63; k < a.nparts; k += 64) s += a.lossp[k];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) {
        const int64_t t = *a.local;
        if (a.loss_trace) a.loss_trace[t] = s * a.inv_b;
        *a.local = t + 1;
        if (a.step) {
            const int64_t n = *a.step;
            const double done = (double)n;
            const double tt = done + 1.0;
            a.coef[0] = (float)(1.0 - pow((double)a.ad.b1, tt));
            a.coef[1] = (float)(1.0 - pow((double)a.ad.b2, tt));
            float lr = a.ad.lr;
            if (a.ad.decay_steps > 0.0) {
                const double x = fmin(done / a.ad.decay_steps, 1.0);
                lr = (float)(a.ad.lr * (a.ad.final_frac + (1.0 - a.ad.final_frac) * 0.5 * (1.0 + cospi(x))));
            }
            a.coef[2] = lr;
            *a.step = n + 1;
        }
    }
}

__global__ __launch_bounds__(256) void wgrad_group_kernel(WgradGroup g) {
    const int b = blockIdx.x;
    if (b < g.gemm_blocks) {
        const int k = b >= g.job[2].first ? 2 : (b >= g.job[1].first ? 1 : 0);
        const WgradJob j = k == 0 ? g.job[0] : (k == 1 ? g.job[1] : g.job[2]);
        int local = b - j.first;
        const int bx = local % j.tx;
        local /= j.tx;
        const int by = local % j.ty, bz = local / j.ty;
        gemm_nt_tile<kEpiOutF32>(j.A, j.B, j.M, j.N, j.R, j.lda, j.ldb, nullptr, nullptr, nullptr, nullptr, j.partial,
                                 j.chunk, bx, by, bz);
    } else if (b < g.gemm_blocks + 3 * 256) {
        bias_grad_unit(g.g1, g.g2, g.g3, g.B, g.bgrad, b - g.gemm_blocks);
    } else if (threadIdx.x < 64) {
        advance_unit(g.adv);
    }
}

// ------------------------------------------------------------ update --
__global__ __launch_bounds__(256) void adam_kernel(MlpView w, SplitParts sp, const float *__restrict__ bgrad, AdamSpec ad,
                                                   const float *__restrict__ coef, float *__restrict__ grad) {
    adam_unit(w, sp, bgrad, ad, coef, grad, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(64) void advance_kernel(AdvanceJob a) { advance_unit(a); }

__global__ void set_i64_kernel(int64_t *p, int64_t v) { *p = v; }

// Glorot-uniform weights: element e of W_l[out][in] takes word e mod 4 of
// Philox block (e div 4, l, 0, tag 5), w = (2u - 1) sqrt(6 / (in + out)) in
// FP32; zero biases and moments; zero step count.
__global__ __launch_bounds__(256) void init_weights_kernel(MlpView w, Key key, float s0, float s1, float s2) {
#pragma clang fp contract(off)
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e == 0) *w.step = 0;
    if (e >= MlpParams::count()) return;
    int l = 0;
    if (e >= MlpParams::w_off(2)) l = 2;
    else if (e >= MlpParams::w_off(1)) l = 1;
    const int in = MlpParams::in(l), out = MlpParams::out(l);
    const int64_t local = e - MlpParams::w_off(l);
    float p = 0.0f;
    if (local < (int64_t)in * out) {
        const uint4 q = philox((uint32_t)(local >> 2), (uint32_t)l, 0, kTagInit, key);
        const uint32_t word = (local & 3) == 0 ? q.x : (local & 3) == 1 ? q.y : (local & 3) == 2 ? q.z : q.w;
        const float scale = l == 0 ? s0 : (l == 1 ? s1 : s2);
        p = (2.0f * unit_f32(word) - 1.0f) * scale;
        const int o = (int)(local / in), i = (int)(local % in);
        const uint16_t h = f32_to_bf16(p);
        w.wt[MlpParams::bf16_w_off(l) + local] = h;
        w.w[MlpParams::bf16_w_off(l) + (int64_t)i * out + o] = h;
        w.wtf[MlpParams::bf16_w_off(l) + frag_index(o, i, in)] = h;
        w.wf[MlpParams::bf16_w_off(l) + frag_index(i, o, out)] = h;
    }
    w.master[e] = p;
    w.m[e] = 0.0f;
    w.v[e] = 0.0f;
}

// -------------------------------------------------------------- decode --
// FP64 proposal parameters from network output column 0 (log-scales raised
// by log_widen).
//   POLY: {log-softmax of the degree logits [4], log-softmax of the mixture
//          logits [8], mean[4][8][5], lsd[4][8][5]} (slots j >= n zero).
//   GMM:  {log-softmax of the mixture logits [8], mean[8][d], lsd[8][d]}.
__global__ __launch_bounds__(64) void decode_kernel(int model, int K, const float *__restrict__ o_col, int ld,
                                                    double log_widen, double *__restrict__ q) {
    const int lane = threadIdx.x;
    auto O = [&](int k) { return (double)o_col[(size_t)k * ld]; };
    auto logsoftmax = [&](int base, int n, double *dst) {
        double m = -INFINITY;
        for (int k = 0; k < n; ++k) m = fmax(m, O(base + k));
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += exp(O(base + k) - m);
        const double ls = log(s);
        for (int k = 0; k < n; ++k) dst[k] = O(base + k) - m - ls;
    };
    if (model == PPL_MODEL_POLY) {
        if (lane == 0) logsoftmax(0, 4, q);
        if (lane == 1) logsoftmax(4, 8, q + 4);
        for (int e = lane; e < 160; e += 64) {
            const int n = 2 + e / 40, m = (e / 5) % 8, j = e % 5;
            const int off = poly_head_off(n);
            q[12 + e] = j < n ? 10.0 * O(off + m * n + j) : 0.0;
            q[172 + e] = j < n ? 5.0 * tanh(O(off + 8 * n + m * n + j) / 5.0) + log_widen : 0.0;
        }
    } else {
        const int d = 2 * K - 1;
        if (lane == 0) logsoftmax(0, 8, q);
        for (int e = lane; e < 8 * d; e += 64) {
            q[8 + e] = 5.0 * O(8 + e);
            q[8 + 8 * d + e] = 5.0 * tanh(O(8 + 8 * d + e) / 5.0) + log_widen;
        }
    }
}

// ---------------------------------------------------------------- host --
static size_t a256(size_t v) { return align_up(v, 256); }

size_t train_ws_bytes(int B) {
    int nc[3], ch[3];
    mlp_split_plan(kMlpHid, kMlpIn, B, &nc[0], &ch[0]);
    mlp_split_plan(kMlpHid, kMlpHid, B, &nc[1], &ch[1]);
    mlp_split_plan(kMlpOut, kMlpHid, B, &nc[2], &ch[2]);
    const size_t bB = (size_t)B;
    size_t n = 0;
    n += 2 * a256(bB * kSummaryDim * 2);                 // x row / col
    n += a256(bB * kThetaStride * 8);                    // theta
    n += 4 * a256(bB * kMlpHid * 2);                     // h1, h2 row / col
    n += a256(bB * kMlpOut * 4);                         // o_col
    n += 5 * a256(bB * kMlpOut * 2);                     // do row/col, dh2 row/col, dh1 col
    n += a256((size_t)nc[0] * kMlpHid * kMlpIn * 4);
    n += a256((size_t)nc[1] * kMlpHid * kMlpHid * 4);
    n += a256((size_t)nc[2] * kMlpOut * kMlpHid * 4);
    n += a256(3 * 256 * 4);                              // bgrad
    n += a256((bB / kHeadPairs + 1) * 8);                // loss partials
    n += 256;                                            // local counter
    return n;
}

TrainBufs train_bufs(void *ws, int B) {
    TrainBufs t{};
    t.B = B;
    mlp_split_plan(kMlpHid, kMlpIn, B, &t.nchunks[0], &t.chunk[0]);
    mlp_split_plan(kMlpHid, kMlpHid, B, &t.nchunks[1], &t.chunk[1]);
    mlp_split_plan(kMlpOut, kMlpHid, B, &t.nchunks[2], &t.chunk[2]);
    char *p = (char *)ws;
    const size_t bB = (size_t)B;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += a256(bytes);
        return (void *)r;
    };
    t.x_row = (uint16_t *)take(bB * kSummaryDim * 2);
    t.x_col = (uint16_t *)take(bB * kSummaryDim * 2);
    t.theta = (double *)take(bB * kThetaStride * 8);
    t.h1_row = (uint16_t *)take(bB * kMlpHid * 2);
    t.h1_col = (uint16_t *)take(bB * kMlpHid * 2);
    t.h2_row = (uint16_t *)take(bB * kMlpHid * 2);
    t.h2_col = (uint16_t *)take(bB * kMlpHid * 2);
    t.o_col = (float *)take(bB * kMlpOut * 4);
    t.do_row = (uint16_t *)take(bB * kMlpOut * 2);
    t.do_col = (uint16_t *)take(bB * kMlpOut * 2);
    t.dh2_row = (uint16_t *)take(bB * kMlpOut * 2);
    t.dh2_col = (uint16_t *)take(bB * kMlpOut * 2);
    t.dh1_col = (uint16_t *)take(bB * kMlpOut * 2);
    t.part[0] = (float *)take((size_t)t.nchunks[0] * kMlpHid * kMlpIn * 4);
    t.part[1] = (float *)take((size_t)t.nchunks[1] * kMlpHid * kMlpHid * 4);
    t.part[2] = (float *)take((size_t)t.nchunks[2] * kMlpOut * kMlpHid * 4);
    t.bgrad = (float *)take(3 * 256 * 4);
    t.lossp = (double *)take((bB / kHeadPairs + 1) * 8);
    t.local = (int64_t *)take(64);
    t.coef = (float *)(t.local + 4);
    return t;
}

int launch_forward(const MlpView &w, const TrainBufs &b, bool keep_cols, hipStream_t st) {
    const int epi = kEpiBias | kEpiRelu | kEpiOutRow | (keep_cols ? kEpiOutCol : 0);
    if (int rc = mlp_gemm(b.x_row, w.wt + MlpParams::bf16_w_off(0), b.B, kMlpHid, kMlpIn, kMlpIn, kMlpIn, epi,
                          w.master + MlpParams::b_off(0), nullptr, b.h1_row, b.h1_col, nullptr, st))
        return rc;
    if (int rc = mlp_gemm(b.h1_row, w.wt + MlpParams::bf16_w_off(1), b.B, kMlpHid, kMlpHid, kMlpHid, kMlpHid, epi,
                          w.master + MlpParams::b_off(1), nullptr, b.h2_row, b.h2_col, nullptr, st))
        return rc;
    return mlp_gemm(b.h2_row, w.wt + MlpParams::bf16_w_off(2), b.B, kMlpOut, kMlpHid, kMlpHid, kMlpHid,
                    kEpiBias | kEpiOutF32Col, w.master + MlpParams::b_off(2), nullptr, nullptr, nullptr, b.o_col, st);
}

int launch_head_backward(int model, int K, const MlpView &w, const TrainBufs &b, hipStream_t st) {
    const int B = b.B;
    const float inv_b = 1.0f / (float)B;
    {
        KernelTimer timer("head_kernel", st);
        if (model == PPL_MODEL_POLY)
            hipLaunchKernelGGL(head_kernel<PPL_MODEL_POLY>, dim3(B / kHeadPairs), dim3(256), 0, st, b.o_col, B,
                               b.theta, K, inv_b, b.do_row, b.do_col, b.lossp);
        else
            hipLaunchKernelGGL(head_kernel<PPL_MODEL_GMM>, dim3(B / kHeadPairs), dim3(256), 0, st, b.o_col, B,
                               b.theta, K, inv_b, b.do_row, b.do_col, b.lossp);
        timer.stop();
        PPL_LAUNCH_CHECK("head_kernel");
    }
    // layer 3: dW3 = dO^T H2, dH2 = (dO W3) * [H2 > 0]
    if (int rc = mlp_gemm_splitr(b.do_col, b.h2_col, kMlpOut, kMlpHid, B, B, B, b.chunk[2], b.part[2], st)) return rc;
    if (int rc = mlp_gemm(b.do_row, w.w + MlpParams::bf16_w_off(2), B, kMlpHid, kMlpOut, kMlpOut, kMlpOut,
                          kEpiMaskRow | kEpiOutRow | kEpiOutCol, nullptr, b.h2_row, b.dh2_row, b.dh2_col, nullptr, st))
        return rc;
    // layer 2: dW2 = dH2^T H1, dH1 = (dH2 W2) * [H1 > 0]
    if (int rc = mlp_gemm_splitr(b.dh2_col, b.h1_col, kMlpHid, kMlpHid, B, B, B, b.chunk[1], b.part[1], st)) return rc;
    if (int rc = mlp_gemm(b.dh2_row, w.w + MlpParams::bf16_w_off(1), B, kMlpHid, kMlpHid, kMlpHid, kMlpHid,
                          kEpiMaskRow | kEpiOutCol, nullptr, b.h1_row, nullptr, b.dh1_col, nullptr, st))
        return rc;
    // layer 1: dW1 = dH1^T X
    if (int rc = mlp_gemm_splitr(b.dh1_col, b.x_col, kMlpHid, kMlpIn, B, B, B, b.chunk[0], b.part[0], st)) return rc;
    hipLaunchKernelGGL(bias_grad_kernel, dim3(3 * 256), dim3(256), 0, st, b.dh1_col, b.dh2_col, b.do_col, B, b.bgrad);
    PPL_LAUNCH_CHECK("bias_grad_kernel");
    return PPL_OK;
}

// The fused pass (forward, head, input gradients) then the weight-gradient
// products and bias sums of launch_head_backward.
int launch_fused_pass(int model, int K, const MlpView &w, const TrainBufs &b, const AdvanceJob &adv, hipStream_t st) {
    const int B = b.B;
    if (B % kFuseRows) return fail(PPL_E_ARG, "batch %d is not a multiple of %d", B, kFuseRows);
    const float inv_b = 1.0f / (float)B;
    {
        KernelTimer timer("fused_pass_kernel", st);
        if (model == PPL_MODEL_POLY)
            hipLaunchKernelGGL(fused_pass_kernel<PPL_MODEL_POLY>, dim3(B / kFuseRows), dim3(256), 0, st, w, b, K, inv_b);
        else
            hipLaunchKernelGGL(fused_pass_kernel<PPL_MODEL_GMM>, dim3(B / kFuseRows), dim3(256), 0, st, w, b, K, inv_b);
        timer.stop();
        PPL_LAUNCH_CHECK("fused_pass_kernel");
    }
    // the weight-gradient products and bias sums, grouped in one launch
    WgradGroup g{};
    const uint16_t *As[3] = {b.do_col, b.dh2_col, b.dh1_col}, *Bs[3] = {b.h2_col, b.h1_col, b.x_col};
    const int Ms[3] = {kMlpOut, kMlpHid, kMlpHid}, Ns[3] = {kMlpHid, kMlpHid, kMlpIn}, layer[3] = {2, 1, 0};
    int first = 0;
    for (int k = 0; k < 3; ++k) {
        const int l = layer[k], chunk = b.chunk[l];
        if (Ms[k] % kGemmTile || Ns[k] % kGemmTile || B % 32 || chunk % 32 || chunk <= 0)
            return fail(PPL_E_ARG, "split GEMM shape %d x %d x %d / %d not tile-aligned", Ms[k], Ns[k], B, chunk);
        WgradJob &j = g.job[k];
        j.A = As[k];
        j.B = Bs[k];
        j.partial = b.part[l];
        j.M = Ms[k];
        j.N = Ns[k];
        j.R = B;
        j.lda = B;
        j.ldb = B;
        j.chunk = chunk;
        j.tx = Ns[k] / kGemmTile;
        j.ty = Ms[k] / kGemmTile;
        j.first = first;
        first += j.tx * j.ty * ((B + chunk - 1) / chunk);
    }
    g.gemm_blocks = first;
    g.g1 = b.dh1_col;
    g.g2 = b.dh2_col;
    g.g3 = b.do_col;
    g.B = B;
    g.bgrad = b.bgrad;
    g.adv = adv;
    {
        KernelTimer timer("wgrad_group_kernel", st);
        hipLaunchKernelGGL(wgrad_group_kernel, dim3((unsigned)(first + 3 * 256 + 1)), dim3(256), 0, st, g);
        timer.stop();
        PPL_LAUNCH_CHECK("wgrad_group_kernel");
    }
    return PPL_OK;
}

int launch_update(const MlpView &w, const TrainBufs &b, const AdamSpec &ad, float *grad, hipStream_t st) {
    const SplitParts sp = split_parts(b);
    const int blocks = (int)((MlpParams::count() + 255) / 256);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, st, w, sp, (const float *)b.bgrad, ad,
                       (const float *)b.coef, grad);
    PPL_LAUNCH_CHECK("adam_kernel");
    return PPL_OK;
}

AdvanceJob advance_job(int64_t *step, const TrainBufs &b, const AdamSpec &ad, double *loss_trace) {
    AdvanceJob a{};
    a.step = step;
    a.local = b.local;
    a.lossp = b.lossp;
    a.nparts = b.B / kHeadPairs;
    a.inv_b = 1.0 / (double)b.B;
    a.loss_trace = loss_trace;
    a.ad = ad;
    a.coef = b.coef;
    return a;
}

int launch_advance(const AdvanceJob &adv, hipStream_t st) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, st, adv);
    PPL_LAUNCH_CHECK("advance_kernel");
    return PPL_OK;
}

int launch_set_i64(int64_t *p, int64_t v, hipStream_t st) {
    hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(1), 0, st, p, v);
    PPL_LAUNCH_CHECK("set_i64_kernel");
    return PPL_OK;
}

int launch_init_weights(void *weights, uint64_t seed, hipStream_t st) {
    const MlpView w = mlp_view(weights);
    float s[3];
    for (int l = 0; l < 3; ++l) s[l] = (float)sqrt(6.0 / (double)(MlpParams::in(l) + MlpParams::out(l)));
    const int blocks = (int)((MlpParams::count() + 255) / 256);
    hipLaunchKernelGGL(init_weights_kernel, dim3(blocks), dim3(256), 0, st, w, make_key(seed), s[0], s[1], s[2]);
    PPL_LAUNCH_CHECK("init_weights_kernel");
    return PPL_OK;
}

int launch_decode(int model, int K, const float *o_col, int ld, double log_widen, double *q, hipStream_t st) {
    hipLaunchKernelGGL(decode_kernel, dim3(1), dim3(64), 0, st, model, K, o_col, ld, log_widen, q);
    PPL_LAUNCH_CHECK("decode_kernel");
    return PPL_OK;
}

}  // namespace ppl
