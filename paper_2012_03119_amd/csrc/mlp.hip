// Kernels and entry points of the clause-priority network (mlp.h): batched
// inference, the gradient of the mean binary cross-entropy, and Adam.
//
// Gradient: a workgroup of 64 lanes takes 32 samples.  Each of the first 32
// lanes runs one sample forward and backward and leaves its activations and
// deltas in LDS (rows padded to 65 floats, so that the lanes' row writes fall in
// different banks); then lane t accumulates column t of every weight gradient
// over the 32 samples (the sample's activation is read by all lanes at once, a
// broadcast).  Each workgroup writes one partial gradient row; a second kernel
// sums the rows in a fixed order, so the result does not depend on scheduling.
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

namespace gss {

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ p, const float *__restrict__ x,
                                                     uint32_t n, float *__restrict__ out) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float xv[kFeat];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) xv[k] = x[(uint64_t)s * kFeat + k];
    out[s] = sigmoidf_(mlp_logit(p, xv));
}

__global__ __launch_bounds__(64) void k_mlp_grad(const float *__restrict__ p, const float *__restrict__ x,
                                                 const float *__restrict__ y, const uint32_t *__restrict__ order,
                                                 uint64_t first, uint32_t n, float inv_n, float *__restrict__ partials) {
    constexpr int B = kGradSamples, LD = kHid + 1;
    __shared__ float sx[B][kFeat + 1];
    __shared__ float sh1[B][LD], sh2[B][LD], sdz2[B][LD], sdz1[B][LD];
    __shared__ float sdz3[B], sloss[B];
    const uint32_t t = threadIdx.x;
    if (t < B) {
        const uint64_t s = (uint64_t)blockIdx.x * B + t;
        const bool ok = s < n;
        float xv[kFeat], yv = 0.f;
        if (ok) {
            const uint64_t row = order ? order[first + s] : first + s;
#pragma unroll
            for (int k = 0; k < kFeat; ++k) xv[k] = x[row * kFeat + k];
            yv = y[row];
        } else {
#pragma unroll
            for (int k = 0; k < kFeat; ++k) xv[k] = 0.f;
        }
        float h1[kHid];
        mlp_layer1(p, xv, h1);
        float z3 = p[kOffB3];
        float h2[16];
#define GSS_MLP_CHUNK(C)                                                        \
        mlp_layer2_chunk<C>(p, h1, h2);                                         \
        _Pragma("unroll") for (int k = 0; k < 16; ++k) {                        \
            sh2[t][C + k] = h2[k];                                              \
            z3 = fmaf(h2[k], p[kOffW3 + C + k], z3);                            \
        }
        GSS_MLP_CHUNK(0)
        GSS_MLP_CHUNK(16)
        GSS_MLP_CHUNK(32)
        GSS_MLP_CHUNK(48)
#undef GSS_MLP_CHUNK
        const float dz3 = ok ? (sigmoidf_(z3) - yv) * inv_n : 0.f;
        sdz3[t] = dz3;
        sloss[t] = ok ? bce_logit(z3, yv) * inv_n : 0.f;
        float dz2[kHid];
#pragma unroll
        for (int j = 0; j < kHid; ++j) {
            dz2[j] = sh2[t][j] > 0.f ? dz3 * p[kOffW3 + j] : 0.f;
            sdz2[t][j] = dz2[j];
        }
#pragma unroll
        for (int i = 0; i < kHid; ++i) {
            float a = 0.f;
#pragma unroll
            for (int j = 0; j < kHid; ++j) a = fmaf(dz2[j], p[kOffW2 + i * kHid + j], a);
            sdz1[t][i] = h1[i] > 0.f ? a : 0.f;
            sh1[t][i] = h1[i];
        }
#pragma unroll
        for (int k = 0; k < kFeat; ++k) sx[t][k] = xv[k];
    }
    __syncthreads();
    float gw2[kHid], gw1[kFeat];
#pragma unroll
    for (int i = 0; i < kHid; ++i) gw2[i] = 0.f;
#pragma unroll
    for (int k = 0; k < kFeat; ++k) gw1[k] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, gl = 0.f;
    for (int s = 0; s < B; ++s) {
        const float d2 = sdz2[s][t], d1 = sdz1[s][t];
#pragma unroll
        for (int i = 0; i < kHid; ++i) gw2[i] = fmaf(sh1[s][i], d2, gw2[i]);
#pragma unroll
        for (int k = 0; k < kFeat; ++k) gw1[k] = fmaf(sx[s][k], d1, gw1[k]);
        gb1 += d1;
        gb2 += d2;
        gw3 = fmaf(sdz3[s], sh2[s][t], gw3);
        gb3 += sdz3[s];
        gl += sloss[s];
    }
    float *out = partials + (uint64_t)blockIdx.x * (kParams + 1);
#pragma unroll
    for (int i = 0; i < kHid; ++i) out[kOffW2 + i * kHid + t] = gw2[i];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) out[kOffW1 + k * kHid + t] = gw1[k];
    out[kOffB1 + t] = gb1;
    out[kOffB2 + t] = gb2;
    out[kOffW3 + t] = gw3;
    if (t == 0) {
        out[kOffB3] = gb3;
        out[kParams] = gl;
    }
}

// grad[i] = sum over rows of partials[row][i], rows in order; entry kParams is the loss.
__global__ void k_mlp_reduce(const float *__restrict__ partials, uint32_t rows, float *__restrict__ grad,
                             float *__restrict__ loss) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > (uint32_t)kParams) return;
    float a = 0.f;
    for (uint32_t r = 0; r < rows; ++r) a += partials[(uint64_t)r * (kParams + 1) + i];
    if (i < (uint32_t)kParams)
        grad[i] = a;
    else
        *loss = a;
}

__global__ void k_mlp_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, float lr, float beta1, float beta2, float eps, float c1, float c2) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)kParams) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

MlpWork &mlp_work(Ctx &c) {
    if (!c.mlp) {
        auto w = std::make_unique<MlpWork>();
        w->params = (float *)c.dalloc(kParams * 4);
        w->m = (float *)c.dalloc(kParams * 4);
        w->v = (float *)c.dalloc(kParams * 4);
        w->grad = (float *)c.dalloc(kParams * 4);
        w->loss = (float *)c.dalloc(256);
        GSS_HIP(hipHostMalloc((void **)&w->h_loss, 256, hipHostMallocDefault));
        c.mlp = w.release();
    }
    return *c.mlp;
}

void mlp_release(Ctx &c) {
    MlpWork *w = c.mlp;
    if (!w) return;
    c.dfree(w->params);
    c.dfree(w->m);
    c.dfree(w->v);
    c.dfree(w->grad);
    c.dfree(w->partials);
    c.dfree(w->loss);
    c.dfree(w->stage);
    if (w->h_loss) (void)hipHostFree(w->h_loss);
    delete w;
    c.mlp = nullptr;
}

char *mlp_stage(Ctx &c, MlpWork &w, size_t bytes) {
    if (bytes > w.stage_bytes) {
        c.sync();  // queued work may still read the old buffer
        c.dfree(w.stage);
        w.stage = nullptr;
        w.stage_bytes = 0;
        const size_t want = std::max<size_t>(bytes, (size_t)1 << 20);
        w.stage = (char *)c.dalloc(want);
        w.stage_bytes = want;
    }
    return w.stage;
}

void mlp_queue_grad(Ctx &c, MlpWork &w, const float *x, const float *y, const uint32_t *order, uint64_t first,
                    uint32_t n) {
    const uint32_t blocks = (n + kGradSamples - 1) / kGradSamples;
    if (blocks > w.partial_rows) {
        c.sync();
        c.dfree(w.partials);
        w.partials = nullptr;
        w.partial_rows = 0;
        const uint32_t rows = std::max<uint32_t>(blocks, 64);
        w.partials = (float *)c.dalloc((size_t)rows * (kParams + 1) * 4);
        w.partial_rows = rows;
    }
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(64), 0, c.stream, w.params, x, y, order, first, n, 1.f / n,
                       w.partials);
    GSS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 1 + 255) / 256), dim3(256), 0, c.stream, w.partials, blocks,
                       w.grad, w.loss);
    GSS_HIP(hipGetLastError());
}

void mlp_queue_adam(Ctx &c, MlpWork &w, float lr, float beta1, float beta2, float eps) {
    w.step++;
    const double c1 = 1.0 - std::pow((double)beta1, (double)w.step);
    const double c2 = 1.0 - std::pow((double)beta2, (double)w.step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, c.stream, w.params, w.grad, w.m, w.v,
                       lr, beta1, beta2, eps, (float)c1, (float)c2);
    GSS_HIP(hipGetLastError());
}

// Queues the upload of host parameters into w.params through the upload ring.
static void upload_params(Ctx &c, MlpWork &w, const float *params) {
    const Ctx::Staged st = c.stage_upload(kParams * 4);
    std::memcpy(st.h, params, kParams * 4);
    GSS_HIP(hipMemcpyAsync(w.params, st.h, kParams * 4, hipMemcpyHostToDevice, c.stream));
    c.stage_done(st);
}

// A device view of an input array (host arrays are copied to the stage at `off`).
static const char *device_input(Ctx &c, char *stage, size_t off, const void *p, size_t bytes) {
    if (is_device_pointer(p)) return (const char *)p;
    GSS_HIP(hipMemcpyAsync(stage + off, p, bytes, hipMemcpyHostToDevice, c.stream));
    return stage + off;
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace gss

using namespace gss;

extern "C" gss_status gss_mlp_forward(gss_ctx *ctx, const float *params, const float *x, uint32_t n, float *out) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(params && x && out, GSS_ERR_INVALID_ARG, "null argument");
    if (n == 0) return GSS_OK;
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    MlpWork &w = mlp_work(c);
    upload_params(c, w, params);
    const size_t xb = round256((size_t)n * kFeat * 4), ob = round256((size_t)n * 4);
    c.sync();  // the stage may be replaced: nothing queued reads it
    char *st = mlp_stage(c, w, xb + ob);
    const float *dx = (const float *)device_input(c, st, 0, x, (size_t)n * kFeat * 4);
    const bool dev_out = is_device_pointer(out);
    float *dout = dev_out ? out : (float *)(st + xb);
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, c.stream, w.params, dx, n, dout);
    GSS_HIP(hipGetLastError());
    if (!dev_out) GSS_HIP(hipMemcpyAsync(out, dout, (size_t)n * 4, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    GSS_API_END
}

extern "C" gss_status gss_mlp_loss_grad(gss_ctx *ctx, const float *params, const float *x, const float *y, uint32_t n,
                                        float *out_loss, float *out_grad) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(params && x && y && out_loss && out_grad, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(n >= 1, GSS_ERR_INVALID_ARG, "n must be at least 1");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    MlpWork &w = mlp_work(c);
    upload_params(c, w, params);
    const size_t xb = round256((size_t)n * kFeat * 4), yb = round256((size_t)n * 4);
    c.sync();
    char *st = mlp_stage(c, w, xb + yb);
    const float *dx = (const float *)device_input(c, st, 0, x, (size_t)n * kFeat * 4);
    const float *dy = (const float *)device_input(c, st, xb, y, (size_t)n * 4);
    mlp_queue_grad(c, w, dx, dy, nullptr, 0, n);
    GSS_HIP(hipMemcpyAsync(w.h_loss, w.loss, 4, hipMemcpyDeviceToHost, c.stream));
    GSS_HIP(hipMemcpyAsync(out_grad, w.grad, kParams * 4,
                           is_device_pointer(out_grad) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c.stream));
    c.sync();
    *out_loss = *w.h_loss;
    GSS_API_END
}

extern "C" gss_status gss_mlp_train(gss_ctx *ctx, float *params, const float *x, const float *y, uint32_t n,
                                    const uint32_t *order, uint64_t n_order, const gss_adam_config *cfg,
                                    float *out_losses) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(params && x && y && order && cfg, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(n >= 1 && n_order >= 1, GSS_ERR_INVALID_ARG, "n and n_order must be at least 1");
    GSS_REQUIRE(cfg->batch >= 1, GSS_ERR_INVALID_ARG, "batch must be at least 1");
    GSS_REQUIRE(cfg->lr > 0 && cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1 && cfg->eps > 0,
                GSS_ERR_INVALID_ARG, "Adam settings out of range");
    GSS_REQUIRE(!is_device_pointer(order), GSS_ERR_INVALID_ARG, "order must be a host array");
    for (uint64_t i = 0; i < n_order; ++i)
        GSS_REQUIRE(order[i] < n, GSS_ERR_INVALID_ARG, "order entry beyond n");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    MlpWork &w = mlp_work(c);
    upload_params(c, w, params);
    launch_fill_u32(c, (uint32_t *)w.m, kParams, 0);
    launch_fill_u32(c, (uint32_t *)w.v, kParams, 0);
    w.step = 0;
    const uint64_t steps = (n_order + cfg->batch - 1) / cfg->batch;
    const size_t xb = round256((size_t)n * kFeat * 4), yb = round256((size_t)n * 4), ob = round256(n_order * 4),
                 lb = round256(steps * 4);
    c.sync();
    char *st = mlp_stage(c, w, xb + yb + ob + lb);
    const float *dx = (const float *)device_input(c, st, 0, x, (size_t)n * kFeat * 4);
    const float *dy = (const float *)device_input(c, st, xb, y, (size_t)n * 4);
    GSS_HIP(hipMemcpyAsync(st + xb + yb, order, n_order * 4, hipMemcpyHostToDevice, c.stream));
    const uint32_t *dorder = (const uint32_t *)(st + xb + yb);
    float *dlosses = (float *)(st + xb + yb + ob);
    for (uint64_t k = 0; k < steps; ++k) {
        const uint64_t first = k * cfg->batch;
        const uint32_t nb = (uint32_t)std::min<uint64_t>(cfg->batch, n_order - first);
        mlp_queue_grad(c, w, dx, dy, dorder, first, nb);
        GSS_HIP(hipMemcpyAsync(dlosses + k, w.loss, 4, hipMemcpyDeviceToDevice, c.stream));
        mlp_queue_adam(c, w, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps);
    }
    GSS_HIP(hipMemcpyAsync(params, w.params, kParams * 4, hipMemcpyDeviceToHost, c.stream));
    if (out_losses) GSS_HIP(hipMemcpyAsync(out_losses, dlosses, steps * 4, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    GSS_API_END
}
