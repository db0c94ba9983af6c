// C ABI of the proposal network: parameters, pooling, forward, training step
// and checkpoint state (include/me.h).  All device work is enqueued on the
// caller's stream; parameter and state transfers are synchronous.
#include <math.h>
#include <string.h>

#include "ctx.h"

using namespace me;

namespace me {

namespace {

constexpr int kOffW[4] = {0, 2336, 11584, 20832};
constexpr int kOffB[4] = {2304, 11552, 20800, 21696};

constexpr int kStride[4] = {2, 2, 1, 1};

int out_dim(int l, int n) { return (n + kStride[l] - 1) / kStride[l]; }

struct Dims {
    int h[5], w[5];   // h[0] = Hq (input), h[l+1] = output of layer l
};

Dims dims_of(int Hq, int Wq)
{
    Dims d;
    d.h[0] = Hq;
    d.w[0] = Wq;
    for (int l = 0; l < 4; ++l) {
        d.h[l + 1] = out_dim(l, d.h[l]);
        d.w[l + 1] = out_dim(l, d.w[l]);
    }
    return d;
}

template <typename T>
bool dalloc(T** p, size_t count)
{
    *p = nullptr;
    return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T) + 16) == hipSuccess;
}

int fwd_off(int l)
{
    int o = 0;
    for (int j = 0; j < l; ++j) o += cnn_fwd_packed_size(j);
    return o;
}

int bwd_off(int l)
{
    int o = 0;
    for (int j = 0; j < l; ++j) o += cnn_bwd_packed_size(j);
    return o;
}

me_status ensure_params(me_ctx ctx)
{
    CnnState& c = ctx->cnn;
    if (c.params) return ME_OK;
    if (!dalloc(&c.params, kCnnParams) || !dalloc(&c.m, kCnnParams) || !dalloc(&c.v, kCnnParams) ||
        !dalloc(&c.grads, kCnnParams) || !dalloc(&c.wf, (size_t)fwd_off(4)) || !dalloc(&c.wb, (size_t)bwd_off(4)))
        return fail(ME_E_NOMEM, "proposal network: parameter allocation failed");
    return ME_OK;
}

me_status ensure_acts(me_ctx ctx, int n, int Hq, int Wq)
{
    CnnState& c = ctx->cnn;
    if (n <= c.cap_n && Hq <= c.cap_hq && Wq <= c.cap_wq) return ME_OK;
    const int cn = n > c.cap_n ? n : c.cap_n;
    const int ch = Hq > c.cap_hq ? Hq : c.cap_hq;
    const int cw = Wq > c.cap_wq ? Wq : c.cap_wq;
    const Dims d = dims_of(ch, cw);
    (void)hipFree(c.a0);
    (void)hipFree(c.a1);
    (void)hipFree(c.a2);
    (void)hipFree(c.a3);
    (void)hipFree(c.out);
    (void)hipFree(c.dz4);
    (void)hipFree(c.d3);
    (void)hipFree(c.d2);
    (void)hipFree(c.d1);
    (void)hipFree(c.bl);
    (void)hipFree(c.partial);
    c.partial = nullptr;
    c.partial_cap = 0;
    c.cap_n = c.cap_hq = c.cap_wq = 0;
    size_t part = 0;
    for (int l = 0; l < 4; ++l) {
        const size_t f = cnn_wgrad_partial_floats(l, cnn_wgrad_groups(cn, d.h[l + 1], d.w[l + 1]));
        if (f > part) part = f;
    }
    const size_t p1 = (size_t)d.h[1] * d.w[1], p2 = (size_t)d.h[2] * d.w[2], p3 = (size_t)d.h[3] * d.w[3];
    if (!dalloc(&c.a0, (size_t)d.h[0] * d.w[0] * 8) || !dalloc(&c.a1, cn * p1 * 32) || !dalloc(&c.a2, cn * p2 * 32) ||
        !dalloc(&c.a3, cn * p3 * 32) || !dalloc(&c.out, cn * p3 * 3) || !dalloc(&c.dz4, cn * p3 * 4) ||
        !dalloc(&c.d3, cn * p3 * 32) || !dalloc(&c.d2, cn * p2 * 32) || !dalloc(&c.d1, cn * p1 * 32) ||
        !dalloc(&c.bl, cn * p3) || !dalloc(&c.partial, part))
        return fail(ME_E_NOMEM, "proposal network: activation allocation failed");
    c.partial_cap = part;
    c.cap_n = cn;
    c.cap_hq = ch;
    c.cap_wq = cw;
    return ME_OK;
}

me_status forward_impl(me_ctx ctx, const uint16_t* x, int n, int Hq, int Wq, float* out, hipStream_t st)
{
    CnnState& c = ctx->cnn;
    const Dims d = dims_of(Hq, Wq);
    const uint16_t* in[4] = {x, c.a1, c.a2, c.a3};
    void* outs[4] = {c.a1, c.a2, c.a3, out};
    for (int l = 0; l < 4; ++l) {
        hipError_t e = launch_conv_fwd(l, in[l], c.wf + fwd_off(l), c.params + kOffB[l], outs[l], n, d.h[l], d.w[l],
                                       d.h[l + 1], d.w[l + 1], st);
        if (e != hipSuccess) return hip_fail(e, "proposal network: forward launch");
    }
    return ME_OK;
}

me_status check_net_input(me_ctx ctx, const void* x, int n, int Hq, int Wq)
{
    if (!ctx) return fail(ME_E_INVAL, "proposal network: null context");
    if (!x) return fail(ME_E_INVAL, "proposal network: null input");
    if (reinterpret_cast<uintptr_t>(x) & 15u) return fail(ME_E_INVAL, "proposal network: input must be 16-byte aligned");
    if (n < 1 || n > 4096) return fail(ME_E_INVAL, "proposal network: batch %d not in [1, 4096]", n);
    if (Hq < 1 || Wq < 1 || Hq > 8192 || Wq > 8192) return fail(ME_E_INVAL, "proposal network: bad input size");
    if (!ctx->cnn.loaded) return fail(ME_E_STATE, "proposal network: no parameters set");
    return ME_OK;
}

}  // namespace

void CnnState::release()
{
    void* ptrs[] = {params, m, v, grads, wf, wb, a0, a1, a2, a3, out, dz4, d3, d2, d1, bl, partial};
    for (void* p : ptrs) (void)hipFree(p);
    *this = CnnState();
}

me_status cnn_propose(me_ctx ctx, const me_frame* ref, const me_frame* cur, hipStream_t st)
{
    const int Hq = cur->height / 8, Wq = cur->width / 8;
    me_status s = ensure_acts(ctx, 1, Hq, Wq);
    if (s != ME_OK) return s;
    CnnState& c = ctx->cnn;
    hipError_t e = launch_pool(ref->data, ref->pitch, cur->data, cur->pitch, Hq, Wq, c.a0, st);
    if (e != hipSuccess) return hip_fail(e, "proposal network: pool launch");
    e = launch_cnn_fused(c.a0, c.wf, c.params, c.out, 1, Hq, Wq, nullptr, nullptr, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "proposal network: forward launch");
    return ME_OK;
}

}  // namespace me

extern "C" {

me_status me_cnn_set_params(me_ctx ctx, const float* params, int32_t count, float median_per_sample)
{
    if (!ctx || !params) return fail(ME_E_INVAL, "me_cnn_set_params: null argument");
    if (count != kCnnParams) return fail(ME_E_INVAL, "me_cnn_set_params: expected %d parameters", kCnnParams);
    if (!(median_per_sample >= 0.0f)) return fail(ME_E_INVAL, "me_cnn_set_params: bad median");
    for (int i = 0; i < count; ++i)
        if (!isfinite(params[i])) return fail(ME_E_INVAL, "me_cnn_set_params: parameter %d is not finite", i);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    me_status s = ensure_params(ctx);
    if (s != ME_OK) return s;
    CnnState& c = ctx->cnn;
    if ((e = hipMemcpy(c.params, params, sizeof(float) * count, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(c.m, 0, sizeof(float) * count)) != hipSuccess ||
        (e = hipMemset(c.v, 0, sizeof(float) * count)) != hipSuccess)
        return hip_fail(e, "me_cnn_set_params: copy");
    if ((e = launch_pack(c.params, c.wf, c.wb, nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
        return hip_fail(e, "me_cnn_set_params: pack");
    c.step = 0;
    c.loaded = true;
    ctx->median_per_sample = median_per_sample;
    return ME_OK;
}

me_status me_cnn_get_params(me_ctx ctx, float* params, int32_t count, float* median_per_sample)
{
    if (!ctx || !params) return fail(ME_E_INVAL, "me_cnn_get_params: null argument");
    if (count != kCnnParams) return fail(ME_E_INVAL, "me_cnn_get_params: expected %d parameters", kCnnParams);
    if (!ctx->cnn.loaded) return fail(ME_E_STATE, "me_cnn_get_params: no parameters set");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(params, ctx->cnn.params, sizeof(float) * count, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "me_cnn_get_params: copy");
    if (median_per_sample) *median_per_sample = ctx->median_per_sample;
    return ME_OK;
}

me_status me_cnn_pool(me_ctx ctx, const me_frame* ref, const me_frame* cur, uint16_t* x, void* stream)
{
    (void)ctx;
    me_status s = check_pair(ref, cur);
    if (s != ME_OK) return s;
    if (!x) return fail(ME_E_INVAL, "me_cnn_pool: null output");
    if (reinterpret_cast<uintptr_t>(x) & 15u) return fail(ME_E_INVAL, "me_cnn_pool: output must be 16-byte aligned");
    if ((cur->height % 8) || (cur->width % 8))
        return fail(ME_E_UNSUPPORTED, "me_cnn_pool: frame sides must be divisible by 8");
    hipError_t e = launch_pool(ref->data, ref->pitch, cur->data, cur->pitch, cur->height / 8, cur->width / 8, x,
                               reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_cnn_pool: launch");
    return ME_OK;
}

me_status me_cnn_forward(me_ctx ctx, const uint16_t* x, int32_t n, int32_t Hq, int32_t Wq, float* out, void* stream)
{
    me_status s = check_net_input(ctx, x, n, Hq, Wq);
    if (s != ME_OK) return s;
    if (!out) return fail(ME_E_INVAL, "me_cnn_forward: null output");
    hipError_t e = launch_cnn_fused(x, ctx->cnn.wf, ctx->cnn.params, out, n, Hq, Wq, nullptr, nullptr, nullptr,
                                    reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_cnn_forward: launch");
    return ME_OK;
}

me_status me_cnn_forward_acts(me_ctx ctx, const uint16_t* x, int32_t n, int32_t Hq, int32_t Wq, float* out,
                              uint16_t* a0, uint16_t* a1, uint16_t* a2, void* stream)
{
    me_status s = check_net_input(ctx, x, n, Hq, Wq);
    if (s != ME_OK) return s;
    if (!out || !a0 || !a1 || !a2) return fail(ME_E_INVAL, "me_cnn_forward_acts: null output");
    if ((reinterpret_cast<uintptr_t>(a0) | reinterpret_cast<uintptr_t>(a1) | reinterpret_cast<uintptr_t>(a2)) & 15u)
        return fail(ME_E_INVAL, "me_cnn_forward_acts: activations must be 16-byte aligned");
    hipError_t e = launch_cnn_fused(x, ctx->cnn.wf, ctx->cnn.params, out, n, Hq, Wq, a0, a1, a2,
                                    reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_cnn_forward_acts: launch");
    return ME_OK;
}

me_status me_cnn_train_step(me_ctx ctx, const uint16_t* x, const int16_t* mv, const float* weight, int32_t n,
                            int32_t Hq, int32_t Wq, int32_t radius, int32_t refine_radius, float lr, int32_t update,
                            float* grads, float* loss, void* stream)
{
    me_status s = check_net_input(ctx, x, n, Hq, Wq);
    if (s != ME_OK) return s;
    if (!mv) return fail(ME_E_INVAL, "me_cnn_train_step: null labels");
    if (radius < 0 || radius > 64 || refine_radius < 0 || refine_radius > 8)
        return fail(ME_E_INVAL, "me_cnn_train_step: bad radius");
    if (update && !(lr >= 0.0f && lr < 1.0f)) return fail(ME_E_INVAL, "me_cnn_train_step: bad learning rate");
    s = ensure_acts(ctx, n, Hq, Wq);
    if (s != ME_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CnnState& c = ctx->cnn;
    const Dims d = dims_of(Hq, Wq);
    s = forward_impl(ctx, x, n, Hq, Wq, c.out, st);
    if (s != ME_OK) return s;
    const int nblk = d.h[4] * d.w[4];
    hipError_t e = launch_loss(c.out, mv, weight, n, nblk, radius, refine_radius, c.dz4, c.bl, loss, st);
    if (e != hipSuccess) return hip_fail(e, "me_cnn_train_step: loss");
    // backward: layer 3 (input a3, output grad dz4), then 2, 1, 0
    const uint16_t* xin[4] = {x, c.a1, c.a2, c.a3};
    const uint16_t* dzs[4] = {c.d1, c.d2, c.d3, c.dz4};
    uint16_t* dprev[4] = {nullptr, c.d1, c.d2, c.d3};
    for (int l = 3; l >= 0; --l) {
        e = launch_conv_wgrad(l, xin[l], dzs[l], c.partial, c.grads, n, d.h[l], d.w[l], d.h[l + 1], d.w[l + 1], st);
        if (e != hipSuccess) return hip_fail(e, "me_cnn_train_step: weight gradient");
        if (l > 0) {
            e = launch_conv_dgrad(l, dzs[l], c.wb + bwd_off(l), xin[l], dprev[l], n, d.h[l], d.w[l], d.h[l + 1],
                                  d.w[l + 1], st);
            if (e != hipSuccess) return hip_fail(e, "me_cnn_train_step: input gradient");
        }
    }
    if (grads) {
        e = hipMemcpyAsync(grads, c.grads, sizeof(float) * kCnnParams, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "me_cnn_train_step: gradient copy");
    }
    if (update) {
        c.step += 1;
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = (float)(1.0 / (1.0 - pow(b1, (double)c.step)));
        const float c2 = (float)(1.0 / (1.0 - pow(b2, (double)c.step)));
        e = launch_adamw(c.params, c.grads, c.m, c.v, kCnnParams, lr, (float)b1, (float)b2, 1e-8f, 0.01f, c1, c2, st);
        if (e == hipSuccess) e = launch_pack(c.params, c.wf, c.wb, st);
        if (e != hipSuccess) return hip_fail(e, "me_cnn_train_step: update");
    }
    return ME_OK;
}

int64_t me_cnn_state_bytes(void) { return (int64_t)sizeof(float) * 3 * kCnnParams + 2 * sizeof(int64_t); }

me_status me_cnn_save_state(me_ctx ctx, void* buf, int64_t bytes)
{
    if (!ctx || !buf) return fail(ME_E_INVAL, "me_cnn_save_state: null argument");
    if (bytes != me_cnn_state_bytes()) return fail(ME_E_INVAL, "me_cnn_save_state: buffer must hold %lld bytes",
                                                   (long long)me_cnn_state_bytes());
    if (!ctx->cnn.loaded) return fail(ME_E_STATE, "me_cnn_save_state: no parameters set");
    char* p = static_cast<char*>(buf);
    const size_t nb = sizeof(float) * kCnnParams;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(p, ctx->cnn.params, nb, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(p + nb, ctx->cnn.m, nb, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(p + 2 * nb, ctx->cnn.v, nb, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "me_cnn_save_state: copy");
    int64_t tail[2];
    tail[0] = ctx->cnn.step;
    float med = ctx->median_per_sample;
    tail[1] = 0;
    memcpy(&tail[1], &med, sizeof(float));
    memcpy(p + 3 * nb, tail, sizeof(tail));
    return ME_OK;
}

me_status me_cnn_load_state(me_ctx ctx, const void* buf, int64_t bytes)
{
    if (!ctx || !buf) return fail(ME_E_INVAL, "me_cnn_load_state: null argument");
    if (bytes != me_cnn_state_bytes()) return fail(ME_E_INVAL, "me_cnn_load_state: buffer must hold %lld bytes",
                                                   (long long)me_cnn_state_bytes());
    const char* p = static_cast<const char*>(buf);
    const size_t nb = sizeof(float) * kCnnParams;
    int64_t tail[2];
    memcpy(tail, p + 3 * nb, sizeof(tail));
    float med;
    memcpy(&med, &tail[1], sizeof(float));
    me_status s = me_cnn_set_params(ctx, reinterpret_cast<const float*>(p), kCnnParams, med);
    if (s != ME_OK) return s;
    hipError_t e = hipMemcpy(ctx->cnn.m, p + nb, nb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->cnn.v, p + 2 * nb, nb, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "me_cnn_load_state: copy");
    ctx->cnn.step = tail[0];
    return ME_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Single stages of the network, for checking each kernel in isolation.

namespace me {
namespace {

const int kCinL[4] = {8, 32, 32, 32}, kCoutL[4] = {32, 32, 32, 3};

me_status check_layer(me_ctx ctx, int l, const void* a, const void* b, int n, int H, int W)
{
    if (!ctx) return fail(ME_E_INVAL, "proposal network: null context");
    if (l < 0 || l > 3) return fail(ME_E_INVAL, "proposal network: layer %d not in [0,3]", l);
    if (!a || !b) return fail(ME_E_INVAL, "proposal network: null argument");
    if ((reinterpret_cast<uintptr_t>(a) & 15u) || (reinterpret_cast<uintptr_t>(b) & 15u))
        return fail(ME_E_INVAL, "proposal network: buffers must be 16-byte aligned");
    if (n < 1 || n > 4096 || H < 1 || W < 1 || H > 8192 || W > 8192)
        return fail(ME_E_INVAL, "proposal network: bad batch or size");
    if (!ctx->cnn.loaded) return fail(ME_E_STATE, "proposal network: no parameters set");
    return ME_OK;
}

}  // namespace
}  // namespace me

extern "C" {

me_status me_cnn_layer_forward(me_ctx ctx, int32_t layer, const uint16_t* in, void* out, int32_t n, int32_t H,
                               int32_t W, void* stream)
{
    me_status s = check_layer(ctx, layer, in, out, n, H, W);
    if (s != ME_OK) return s;
    hipError_t e = launch_conv_fwd(layer, in, ctx->cnn.wf + fwd_off(layer), ctx->cnn.params + kOffB[layer], out, n, H,
                                   W, out_dim(layer, H), out_dim(layer, W), reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_cnn_layer_forward: launch");
    return ME_OK;
}

me_status me_cnn_layer_backward(me_ctx ctx, int32_t layer, const uint16_t* x, const uint16_t* dz, uint16_t* dx,
                                float* grads, int32_t n, int32_t H, int32_t W, void* stream)
{
    me_status s = check_layer(ctx, layer, x, dz, n, H, W);
    if (s != ME_OK) return s;
    if (!grads) return fail(ME_E_INVAL, "me_cnn_layer_backward: null gradient buffer");
    if (layer > 0 && !dx) return fail(ME_E_INVAL, "me_cnn_layer_backward: null input-gradient buffer");
    if (dx && (reinterpret_cast<uintptr_t>(dx) & 15u)) return fail(ME_E_INVAL, "me_cnn_layer_backward: misaligned");
    const int Ho = out_dim(layer, H), Wo = out_dim(layer, W);
    // the partial buffer must hold this layer's per-workgroup partials
    const size_t need = cnn_wgrad_partial_floats(layer, cnn_wgrad_groups(n, Ho, Wo));
    CnnState& c = ctx->cnn;
    if (need > c.partial_cap) {
        (void)hipFree(c.partial);
        c.partial = nullptr;
        c.partial_cap = 0;
        if (!dalloc(&c.partial, need)) return fail(ME_E_NOMEM, "me_cnn_layer_backward: allocation failed");
        c.partial_cap = need;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_conv_wgrad(layer, x, dz, c.partial, grads, n, H, W, Ho, Wo, st);
    if (e == hipSuccess && layer > 0)
        e = launch_conv_dgrad(layer, dz, c.wb + bwd_off(layer), x, dx, n, H, W, Ho, Wo, st);
    if (e != hipSuccess) return hip_fail(e, "me_cnn_layer_backward: launch");
    return ME_OK;
}

me_status me_cnn_loss(me_ctx ctx, const float* out, const int16_t* mv, const float* weight, int32_t n, int32_t nblk,
                      int32_t radius, int32_t refine_radius, uint16_t* dz, float* loss, void* stream)
{
    if (!ctx || !out || !mv || !dz || !loss) return fail(ME_E_INVAL, "me_cnn_loss: null argument");
    if (reinterpret_cast<uintptr_t>(dz) & 7u) return fail(ME_E_INVAL, "me_cnn_loss: dz must be 8-byte aligned");
    if (n < 1 || nblk < 1 || radius < 0 || radius > 64 || refine_radius < 0 || refine_radius > 8)
        return fail(ME_E_INVAL, "me_cnn_loss: bad sizes");
    float* bl = nullptr;
    if (hipMalloc(&bl, sizeof(float) * (size_t)n * nblk) != hipSuccess)
        return fail(ME_E_NOMEM, "me_cnn_loss: allocation failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_loss(out, mv, weight, n, nblk, radius, refine_radius, dz, bl, loss, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(bl);
    if (e != hipSuccess) return hip_fail(e, "me_cnn_loss: launch");
    return ME_OK;
}

me_status me_cnn_adamw(me_ctx ctx, const float* grads, float lr, void* stream)
{
    if (!ctx || !grads) return fail(ME_E_INVAL, "me_cnn_adamw: null argument");
    if (!(lr >= 0.0f && lr < 1.0f)) return fail(ME_E_INVAL, "me_cnn_adamw: bad learning rate");
    if (!ctx->cnn.loaded) return fail(ME_E_STATE, "me_cnn_adamw: no parameters set");
    CnnState& c = ctx->cnn;
    c.step += 1;
    const float c1 = (float)(1.0 / (1.0 - pow(0.9, (double)c.step)));
    const float c2 = (float)(1.0 / (1.0 - pow(0.999, (double)c.step)));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_adamw(c.params, grads, c.m, c.v, kCnnParams, lr, 0.9f, 0.999f, 1e-8f, 0.01f, c1, c2, st);
    if (e == hipSuccess) e = launch_pack(c.params, c.wf, c.wb, st);
    if (e != hipSuccess) return hip_fail(e, "me_cnn_adamw: launch");
    return ME_OK;
}

}  // extern "C"
