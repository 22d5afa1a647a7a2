// adam.h -- the per-parameter Adam update of the proposal network, shared by
// the update launch and the grouped launch that also simulates the next batch.
#pragma once

#include "mlp.h"
#include "proposal.h"

namespace ppl {

struct SplitParts {
    const float *p[3];
    int nc[3];
};

inline SplitParts split_parts(const TrainBufs &b) {
    SplitParts sp;
    for (int l = 0; l < 3; ++l) {
        sp.p[l] = b.part[l];
        sp.nc[l] = b.nchunks[l];
    }
    return sp;
}

// Gradient of parameter e: weights sum their split-R partials in chunk order,
// biases come from bgrad.  grad != null: store it; else one Adam step with
// the bias corrections and learning rate of coef (left by the step's
// bookkeeping) and refresh the BF16 weight layouts.
__device__ __forceinline__ void adam_unit(const MlpView &w, const SplitParts &sp, const float *__restrict__ bgrad,
                                          const AdamSpec &ad, const float *__restrict__ coef,
                                          float *__restrict__ grad, int64_t e) {
    if (e >= MlpParams::count()) return;
    int l = 0;
    if (e >= MlpParams::w_off(2)) l = 2;
    else if (e >= MlpParams::w_off(1)) l = 1;
    const int in = MlpParams::in(l), out = MlpParams::out(l);
    const int64_t local = e - MlpParams::w_off(l);
    const bool is_w = local < (int64_t)in * out;
    float gv;
    if (is_w) {
        const float *p = sp.p[l];
        const int64_t sz = (int64_t)in * out;
        gv = 0.0f;
        // loads in groups of four, the adds in the same order as one at a time
        int c = 0;
        for (; c + 4 <= sp.nc[l]; c += 4) {
            const float x0 = p[(size_t)c * sz + local], x1 = p[(size_t)(c + 1) * sz + local];
            const float x2 = p[(size_t)(c + 2) * sz + local], x3 = p[(size_t)(c + 3) * sz + local];
            gv += x0;
            gv += x1;
            gv += x2;
            gv += x3;
        }
        for (; c < sp.nc[l]; ++c) gv += p[(size_t)c * sz + local];
    } else {
        gv = bgrad[l * 256 + (int)(local - (int64_t)in * out)];
    }
    if (grad) {
        grad[e] = gv;
        return;
    }
    const float bc1 = coef[0], bc2 = coef[1], lr = coef[2];
    const float m = ad.b1 * w.m[e] + (1.0f - ad.b1) * gv;
    const float v = ad.b2 * w.v[e] + (1.0f - ad.b2) * gv * gv;
    const float p = w.master[e] - lr * (m / bc1) / (sqrtf(v / bc2) + ad.eps);
    w.m[e] = m;
    w.v[e] = v;
    w.master[e] = p;
    if (is_w) {
        const int o = (int)(local / in), i = (int)(local % in);
        const uint16_t h = f32_to_bf16(p);
        w.wt[MlpParams::bf16_w_off(l) + local] = h;
        w.w[MlpParams::bf16_w_off(l) + (int64_t)i * out + o] = h;
        w.wtf[MlpParams::bf16_w_off(l) + frag_index(o, i, in)] = h;
        w.wf[MlpParams::bf16_w_off(l) + frag_index(i, o, out)] = h;
    }
}

}  // namespace ppl
