// Device side of the clause-priority network: a 12 -> 64 -> 64 -> 1 perceptron
// with ReLU hidden layers and a sigmoid output, in fp32.  The paper has no such
// network; it motivates the priority by its Section 3.2 (a clause used recently
// is likely to be used again soon) and Section 3.7 (activity-based deletion on
// the GPU).  Parameters are packed as W1[12][64] (input major), b1[64],
// W2[64][64], b2[64], w3[64], b3: 5057 floats.
//
// Every sample is one lane.  The parameters are read at addresses that are the
// same for the whole wavefront, so they come through the scalar data cache into
// SGPRs and each multiply-add takes its weight as a scalar operand.
#pragma once

#include "gss_internal.h"

namespace gss {

constexpr int kFeat = 12;
constexpr int kHid = 64;
constexpr int kHist = 8;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kFeat * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid;
constexpr int kParams = kOffB3 + 1;  // 5057
static_assert(kParams == 5057, "parameter layout");

// First layer: h1 = relu(x W1 + b1).
__device__ inline void mlp_layer1(const float *__restrict__ p, const float (&x)[kFeat], float (&h1)[kHid]) {
#pragma unroll
    for (int j = 0; j < kHid; ++j) {
        float a = p[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kFeat; ++i) a = fmaf(x[i], p[kOffW1 + i * kHid + j], a);
        h1[j] = fmaxf(a, 0.f);
    }
}

// Second layer, 16 outputs at a time: h2[c..c+16) = relu(h1 W2 + b2).
template <int C>
__device__ inline void mlp_layer2_chunk(const float *__restrict__ p, const float (&h1)[kHid], float (&h2)[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) h2[k] = p[kOffB2 + C + k];
#pragma unroll
    for (int i = 0; i < kHid; ++i)
#pragma unroll
        for (int k = 0; k < 16; ++k) h2[k] = fmaf(h1[i], p[kOffW2 + i * kHid + C + k], h2[k]);
#pragma unroll
    for (int k = 0; k < 16; ++k) h2[k] = fmaxf(h2[k], 0.f);
}

// The output logit z3 of one sample.
__device__ inline float mlp_logit(const float *__restrict__ p, const float (&x)[kFeat]) {
    float h1[kHid];
    mlp_layer1(p, x, h1);
    float z3 = p[kOffB3];
    float h2[16];
#define GSS_MLP_CHUNK(C)                                                        \
    mlp_layer2_chunk<C>(p, h1, h2);                                             \
    _Pragma("unroll") for (int k = 0; k < 16; ++k) z3 = fmaf(h2[k], p[kOffW3 + C + k], z3);
    GSS_MLP_CHUNK(0)
    GSS_MLP_CHUNK(16)
    GSS_MLP_CHUNK(32)
    GSS_MLP_CHUNK(48)
#undef GSS_MLP_CHUNK
    return z3;
}

__device__ inline float sigmoidf_(float z) { return 1.f / (1.f + expf(-z)); }

// softplus(z) - y z: the binary cross-entropy of logit z against label y.
__device__ inline float bce_logit(float z, float y) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - y * z; }

// The 12 features of a clause from its raw statistics: length, LBD, age in runs,
// source thread, hit counts of its last 8 tested runs (most recent first).
__device__ inline void clause_features(float (&x)[kFeat], uint32_t len, float lbd, uint32_t age, uint32_t src,
                                       float src_scale, const uint32_t (&hist)[kHist]) {
    x[0] = log1pf((float)len);
    x[1] = log1pf(lbd);
    x[2] = log1pf((float)age);
    x[3] = (float)src * src_scale;
#pragma unroll
    for (int k = 0; k < kHist; ++k) x[4 + k] = log1pf((float)hist[k]);
}

// Host-side workspace of the network's kernels (one per context, grown on demand).
struct MlpWork {
    float *params = nullptr;  // [kParams]
    float *m = nullptr, *v = nullptr, *grad = nullptr;  // Adam moments, reduced gradient
    float *partials = nullptr;  // [blocks][kParams + 1] (the last entry of a row: loss)
    uint32_t partial_rows = 0;
    float *loss = nullptr;      // [1]
    char *stage = nullptr;      // device copies of host inputs
    size_t stage_bytes = 0;
    float *h_loss = nullptr;    // pinned
    uint64_t step = 0;          // Adam steps taken with the current moments
};

constexpr uint32_t kGradSamples = 32;  // samples per workgroup of the gradient kernel

// Queues the gradient of the mean loss over n samples (rows order[first..first+n)
// of x/y, or rows first..first+n when order is null) into w.grad, its loss into
// w.loss; inv_n scales both.
void mlp_queue_grad(Ctx &c, MlpWork &w, const float *x, const float *y, const uint32_t *order, uint64_t first,
                    uint32_t n);
// Queues one Adam step on w.params from w.grad.
void mlp_queue_adam(Ctx &c, MlpWork &w, float lr, float beta1, float beta2, float eps);
MlpWork &mlp_work(Ctx &c);
void mlp_release(Ctx &c);
char *mlp_stage(Ctx &c, MlpWork &w, size_t bytes);

}  // namespace gss
