// C ABI of the library (include/me.h): argument validation, launch planning
// and dispatch to the HIP kernels.  Every check runs before the first HIP
// call, so a rejected call enqueues nothing.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "ctx.h"

using namespace me;

namespace {
thread_local char g_err[512] = "";
}  // namespace

namespace me {

me_status fail(me_status s, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

me_status hip_fail(hipError_t e, const char* what)
{
    return fail(ME_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

me_status check_frame(const me_frame* f, const char* name)
{
    if (!f) return fail(ME_E_INVAL, "%s: null frame", name);
    if (!f->data) return fail(ME_E_INVAL, "%s: null data pointer", name);
    if (f->height < 2 || f->width < 2 || (f->height & 1) || (f->width & 1))
        return fail(ME_E_INVAL, "%s: height and width must be even and >= 2 (got %d x %d)", name, f->height,
                    f->width);
    if (f->pitch < f->width || (f->pitch & 1))
        return fail(ME_E_INVAL, "%s: pitch must be even and >= width (got %lld)", name, (long long)f->pitch);
    if (reinterpret_cast<uintptr_t>(f->data) & 3u) return fail(ME_E_INVAL, "%s: data must be 4-byte aligned", name);
    if (f->height > 65536 || f->width > 65536)
        return fail(ME_E_UNSUPPORTED, "%s: frames above 65536 samples per side are not supported", name);
    return ME_OK;
}

bool block_ok(int B) { return B == 8 || B == 16 || B == 32 || B == 64; }

me_status check_pair(const me_frame* ref, const me_frame* cur)
{
    me_status s = check_frame(ref, "ref");
    if (s != ME_OK) return s;
    s = check_frame(cur, "cur");
    if (s != ME_OK) return s;
    if (ref->height != cur->height || ref->width != cur->width)
        return fail(ME_E_INVAL, "ref and cur sizes differ (%dx%d vs %dx%d)", ref->height, ref->width, cur->height,
                    cur->width);
    return ME_OK;
}

SearchArgs make_args(const me_frame* ref, const me_frame* cur, int B, int R, int limit, const int16_t* pred,
                     int16_t* mv, int32_t* sad)
{
    SearchArgs a{};
    a.ref = reinterpret_cast<const uint32_t*>(ref->data);
    a.cur = reinterpret_cast<const uint32_t*>(cur->data);
    a.ref_pitch = ref->pitch / 2;
    a.cur_pitch = cur->pitch / 2;
    a.block = B;
    a.Hp = cur->height / 2;
    a.Wp = cur->width / 2;
    a.bh = (a.Hp + B - 1) / B;
    a.bw = (a.Wp + B - 1) / B;
    a.R = R;
    a.limit = limit;
    a.pred = pred;
    a.pred_ratio = 1;
    a.pred_bw = a.bw;
    a.step = 1;
    a.mv = mv;
    a.sad = sad;
    a.wpb = 4;
    return a;
}

}  // namespace me

me_ctx_s::~me_ctx_s()
{
    (void)hipFree(pred);
    (void)hipFree(fb);
    (void)hipFree(list);
    (void)hipFree(count);
    cnn.release();
    if (staged) (void)hipEventSynchronize(staged);
    if (graph) (void)hipGraphExecDestroy(graph);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    if (staged) (void)hipEventDestroy(staged);
    (void)hipFree(ptrs_dev);
    (void)hipHostFree(ptrs_host);
    (void)hipFree(qjobs_dev);
    (void)hipHostFree(qjobs_host);
    (void)hipFree(qcount);
    (void)hipFree(pyr_mv[0]);
    (void)hipFree(pyr_mv[1]);
    (void)hipFree(pyr_sad);
    (void)hipFree(tune_mv);
    (void)hipFree(tune_sad);
    (void)hipFree(prn_scratch);
    (void)hipFree(stat);
}

namespace me {

me_status ensure_scratch(me_ctx ctx, size_t nblk)
{
    if (nblk <= ctx->cap_blocks) return ME_OK;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    (void)hipFree(ctx->pred);
    (void)hipFree(ctx->fb);
    (void)hipFree(ctx->list);
    (void)hipFree(ctx->count);
    ctx->pred = nullptr;
    ctx->fb = nullptr;
    ctx->list = nullptr;
    ctx->count = nullptr;
    ctx->cap_blocks = 0;
    if (hipMalloc(&ctx->pred, nblk * 2 * sizeof(int16_t)) != hipSuccess ||
        hipMalloc(&ctx->fb, nblk) != hipSuccess || hipMalloc(&ctx->list, nblk * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&ctx->count, sizeof(int32_t)) != hipSuccess)
        return fail(ME_E_NOMEM, "proposal scratch: device allocation of %zu blocks failed", nblk);
    ctx->cap_blocks = nblk;
    return ME_OK;
}

TileCfg tiles_for(me_ctx ctx, int B, int R, int Hp, int Wp)
{
    if (ctx) {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->tuned.find(std::make_tuple(B, R, Hp, Wp));
        if (it != ctx->tuned.end()) return it->second;
    }
    return default_tiles(B, R);
}

me_status refine_run(const me_frame* ref, const me_frame* cur, const me_params& p, float m, const float* net_out,
                     int16_t* mv, int32_t* sad, uint8_t* fallback, const RefineScratch& w, hipStream_t st)
{
    const int Hp = cur->height / 2, Wp = cur->width / 2;
    const int bh = (Hp + p.block - 1) / p.block, bw = (Wp + p.block - 1) / p.block;
    const int nblk = bh * bw;
    uint8_t* fb = fallback ? fallback : w.fb;

    const double ratio_m = (double)p.sad_ratio * (double)m;
    hipError_t e;
    if (small_search(p.block, p.refine_radius)) {
        // the refine kernel decodes its predictors from the network output
        SearchArgs a = make_args(ref, cur, p.block, p.refine_radius, p.radius, nullptr, mv, sad);
        a.net = net_out;
        e = launch_sad_search(a, default_tiles(p.block, p.refine_radius), nblk, st);
        if (e != hipSuccess) return hip_fail(e, "refine: refine search");
    } else {
        e = launch_decode(net_out, nblk, p.radius, w.pred, st);
        if (e != hipSuccess) return hip_fail(e, "refine: decode");
        SearchArgs a = make_args(ref, cur, p.block, p.refine_radius, p.radius, w.pred, mv, sad);
        e = launch_sad_search(a, default_tiles(p.block, p.refine_radius), nblk, st);
        if (e != hipSuccess) return hip_fail(e, "refine: refine search");
    }
    e = launch_fallback(net_out, sad, bh, bw, Hp, Wp, p.block, p.conf_logit_thresh, ratio_m, fb, w.list, w.count, st);
    if (e != hipSuccess) return hip_fail(e, "refine: fallback");
    SearchArgs f = make_args(ref, cur, p.block, p.radius, p.radius, nullptr, mv, sad);
    f.list = w.list;
    f.list_n = w.count;
    e = launch_sad_search(f, list_tiles(p.block, p.radius), nblk, st);
    if (e != hipSuccess) return hip_fail(e, "refine: fallback search");
    return ME_OK;
}

me_status refine_impl(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params& p, const float* net_out,
                      int16_t* mv, int32_t* sad, uint8_t* fallback, hipStream_t st)
{
    const float m = p.sad_median_per_sample > 0.0f ? p.sad_median_per_sample : ctx->median_per_sample;
    if (!(m > 0.0f)) return fail(ME_E_STATE, "refine: no SAD median (params or loaded weights)");
    const int Hp = cur->height / 2, Wp = cur->width / 2;
    const int bh = (Hp + p.block - 1) / p.block, bw = (Wp + p.block - 1) / p.block;
    me_status s = ensure_scratch(ctx, (size_t)bh * bw);
    if (s != ME_OK) return s;
    const RefineScratch w{ctx->pred, ctx->fb, ctx->list, ctx->count};
    return refine_run(ref, cur, p, m, net_out, mv, sad, fallback, w, st);
}

me_status check_refine_params(const me_params& p)
{
    if (!block_ok(p.block)) return fail(ME_E_UNSUPPORTED, "block %d not in {8,16,32,64}", p.block);
    if (p.radius < 0 || p.radius > 64) return fail(ME_E_INVAL, "radius %d not in [0,64]", p.radius);
    if (p.refine_radius < 0 || p.refine_radius > 8)
        return fail(ME_E_INVAL, "refine radius %d not in [0,8]", p.refine_radius);
    if (!(p.sad_ratio >= 0.0f)) return fail(ME_E_INVAL, "sad_ratio must be >= 0");
    return ME_OK;
}

}  // namespace me

extern "C" {

const char* me_status_string(me_status s)
{
    switch (s) {
    case ME_OK: return "ME_OK";
    case ME_E_INVAL: return "ME_E_INVAL";
    case ME_E_UNSUPPORTED: return "ME_E_UNSUPPORTED";
    case ME_E_HIP: return "ME_E_HIP";
    case ME_E_NOMEM: return "ME_E_NOMEM";
    case ME_E_STATE: return "ME_E_STATE";
    }
    return "ME_E_UNKNOWN";
}

const char* me_last_error(void) { return g_err; }

me_params me_default_params(void)
{
    me_params p;
    p.block = 16;
    p.radius = 32;
    p.step = 1;
    p.mode = ME_MODE_EXHAUSTIVE;
    p.refine_radius = 2;
    p.conf_logit_thresh = 0.0f;
    p.sad_ratio = 1.5f;
    p.sad_median_per_sample = 0.0f;
    return p;
}

me_status me_ctx_create(int32_t device, me_ctx* out)
{
    if (!out) return fail(ME_E_INVAL, "me_ctx_create: null output pointer");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(ME_E_INVAL, "me_ctx_create: device %d not in [0, %d)", device, n);
    // the device address of me_refine_noalloc's fixed scratch, once per device
    me_status s = noalloc_resolve(device);
    if (s != ME_OK) return s;
    me_ctx c = new (std::nothrow) me_ctx_s;
    if (!c) return fail(ME_E_NOMEM, "me_ctx_create: out of host memory");
    c->device = device;
    *out = c;
    return ME_OK;
}

me_status me_ctx_destroy(me_ctx ctx)
{
    if (!ctx) return fail(ME_E_INVAL, "me_ctx_destroy: null context");
    delete ctx;
    return ME_OK;
}

me_status me_estimate(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params* params, int16_t* mv,
                      int32_t* sad, uint8_t* fallback, void* stream)
{
    me_status s = check_pair(ref, cur);
    if (s != ME_OK) return s;
    if (!params) return fail(ME_E_INVAL, "me_estimate: null params");
    if (!mv || !sad) return fail(ME_E_INVAL, "me_estimate: null mv or sad");
    const me_params& p = *params;
    if (!block_ok(p.block)) return fail(ME_E_UNSUPPORTED, "me_estimate: block %d not in {8,16,32,64}", p.block);
    if (p.radius < 0 || p.radius > 64) return fail(ME_E_INVAL, "me_estimate: radius %d not in [0,64]", p.radius);
    if (p.step != 1) return fail(ME_E_UNSUPPORTED, "me_estimate: step %d (only 1 is supported)", p.step);
    if (p.mode != ME_MODE_EXHAUSTIVE && p.mode != ME_MODE_PROPOSAL)
        return fail(ME_E_INVAL, "me_estimate: unknown mode %d", p.mode);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (p.mode == ME_MODE_PROPOSAL) {
        if (!ctx || !ctx->cnn.loaded) return fail(ME_E_STATE, "me_estimate: proposal mode needs loaded weights");
        s = check_refine_params(p);
        if (s != ME_OK) return s;
        if (p.block != 16 || (cur->height % 8) || (cur->width % 8))
            return fail(ME_E_UNSUPPORTED, "me_estimate: proposal mode needs B=16 and frame sides divisible by 8");
        s = cnn_propose(ctx, ref, cur, st);
        if (s != ME_OK) return s;
        return refine_impl(ctx, ref, cur, p, ctx->cnn.out, mv, sad, fallback, st);
    }

    SearchArgs a = make_args(ref, cur, p.block, p.radius, p.radius, nullptr, mv, sad);
    const TileCfg cfg = tiles_for(ctx, p.block, p.radius, a.Hp, a.Wp);
    hipError_t e = launch_sad_search(a, cfg, a.bh * a.bw, st);
    if (e != hipSuccess) return hip_fail(e, "me_estimate: search launch");
    if (fallback) {
        e = launch_fill_u8(fallback, (size_t)a.bh * a.bw, 0, st);
        if (e != hipSuccess) return hip_fail(e, "me_estimate: fallback fill");
    }
    return ME_OK;
}

me_status me_stage_search(me_ctx ctx, const me_frame* ref, const me_frame* cur, int32_t block, int32_t radius,
                          int32_t step, const int16_t* pred, int32_t limit, int16_t* mv, int32_t* sad, void* stream)
{
    me_status s = check_pair(ref, cur);
    if (s != ME_OK) return s;
    if (!mv || !sad) return fail(ME_E_INVAL, "me_stage_search: null mv or sad");
    if (!block_ok(block)) return fail(ME_E_UNSUPPORTED, "me_stage_search: block %d not in {8,16,32,64}", block);
    if (radius < 0 || radius > 64) return fail(ME_E_INVAL, "me_stage_search: radius %d not in [0,64]", radius);
    if (step < 1 || step > 64) return fail(ME_E_INVAL, "me_stage_search: step %d not in [1,64]", step);
    if (limit < 0 || limit > 127) return fail(ME_E_INVAL, "me_stage_search: limit %d not in [0,127]", limit);
    if (step > 1 && !step_supported(block, radius, step))
        return fail(ME_E_UNSUPPORTED, "me_stage_search: window of block %d, radius %d, step %d too wide", block,
                    radius, step);
    SearchArgs a = make_args(ref, cur, block, radius, limit, pred, mv, sad);
    a.step = step;
    const TileCfg cfg = tiles_for(ctx, block, radius, a.Hp, a.Wp);
    hipError_t e = launch_sad_search(a, cfg, a.bh * a.bw, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_stage_search: launch");
    return ME_OK;
}

me_pyramid_cfg me_default_pyramid(void)
{
    me_pyramid_cfg c;
    memset(&c, 0, sizeof c);
    c.n_levels = 2;
    c.block[0] = 32;
    c.block[1] = 16;
    c.n_stages = 3;
    c.radius[0] = 8;
    c.step[0] = 8;
    c.radius[1] = 4;
    c.step[1] = 4;
    c.radius[2] = 2;
    c.step[2] = 1;
    c.limit = 127;
    return c;
}

me_status me_pyramid(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_pyramid_cfg* cfg, int16_t* mv,
                     int32_t* sad, void* stream)
{
    if (!ctx) return fail(ME_E_INVAL, "me_pyramid: null context");
    if (!cfg) return fail(ME_E_INVAL, "me_pyramid: null configuration");
    me_status s = check_pair(ref, cur);
    if (s != ME_OK) return s;
    if (!mv || !sad) return fail(ME_E_INVAL, "me_pyramid: null mv or sad");
    const me_pyramid_cfg& c = *cfg;
    if (c.n_levels < 1 || c.n_levels > 4) return fail(ME_E_INVAL, "me_pyramid: n_levels %d not in [1,4]", c.n_levels);
    if (c.n_stages < 1 || c.n_stages > 4) return fail(ME_E_INVAL, "me_pyramid: n_stages %d not in [1,4]", c.n_stages);
    if (c.limit < 0 || c.limit > 127) return fail(ME_E_INVAL, "me_pyramid: limit %d not in [0,127]", c.limit);
    for (int l = 0; l < c.n_levels; ++l) {
        if (!block_ok(c.block[l])) return fail(ME_E_UNSUPPORTED, "me_pyramid: block %d not in {8,16,32,64}", c.block[l]);
        if (l > 0 && c.block[l - 1] % c.block[l])
            return fail(ME_E_INVAL, "me_pyramid: block %d does not divide %d", c.block[l], c.block[l - 1]);
    }
    for (int k = 0; k < c.n_stages; ++k) {
        if (c.radius[k] < 0 || c.radius[k] > 64) return fail(ME_E_INVAL, "me_pyramid: radius %d not in [0,64]", c.radius[k]);
        if (c.step[k] < 1 || c.step[k] > 64) return fail(ME_E_INVAL, "me_pyramid: step %d not in [1,64]", c.step[k]);
        for (int l = 0; l < c.n_levels; ++l)
            if (c.step[k] > 1 && !step_supported(c.block[l], c.radius[k], c.step[k]))
                return fail(ME_E_UNSUPPORTED, "me_pyramid: window of block %d, radius %d, step %d too wide",
                            c.block[l], c.radius[k], c.step[k]);
    }
    const int Hp = cur->height / 2, Wp = cur->width / 2;
    size_t most = 0;
    for (int l = 0; l < c.n_levels; ++l) {
        const size_t nb = (size_t)((Hp + c.block[l] - 1) / c.block[l]) * ((Wp + c.block[l] - 1) / c.block[l]);
        if (nb > most) most = nb;
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (most > ctx->pyr_cap) {
        (void)hipFree(ctx->pyr_mv[0]);
        (void)hipFree(ctx->pyr_mv[1]);
        (void)hipFree(ctx->pyr_sad);
        ctx->pyr_mv[0] = ctx->pyr_mv[1] = nullptr;
        ctx->pyr_sad = nullptr;
        ctx->pyr_cap = 0;
        if (hipMalloc(&ctx->pyr_mv[0], most * 2 * sizeof(int16_t)) != hipSuccess ||
            hipMalloc(&ctx->pyr_mv[1], most * 2 * sizeof(int16_t)) != hipSuccess ||
            hipMalloc(&ctx->pyr_sad, most * sizeof(int32_t)) != hipSuccess)
            return fail(ME_E_NOMEM, "me_pyramid: scratch allocation failed");
        ctx->pyr_cap = most;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int16_t* prev = nullptr;      // previous stage's vectors
    int prev_block = 0, prev_bw = 0;
    int buf = 0;
    for (int l = 0; l < c.n_levels; ++l) {
        for (int k = 0; k < c.n_stages; ++k) {
            const bool last = l == c.n_levels - 1 && k == c.n_stages - 1;
            int16_t* out_mv = last ? mv : ctx->pyr_mv[buf];
            int32_t* out_sad = last ? sad : ctx->pyr_sad;
            SearchArgs a = make_args(ref, cur, c.block[l], c.radius[k], c.limit, prev, out_mv, out_sad);
            a.step = c.step[k];
            if (prev && k == 0) {                   // parent block's vector
                a.pred_ratio = prev_block / c.block[l];
                a.pred_bw = prev_bw;
            }
            e = launch_sad_search(a, tiles_for(ctx, a.block, a.R, a.Hp, a.Wp), a.bh * a.bw, st);
            if (e != hipSuccess) return hip_fail(e, "me_pyramid: stage launch");
            prev = out_mv;
            prev_block = c.block[l];
            prev_bw = a.bw;
            buf ^= 1;
        }
    }
    return ME_OK;
}

namespace {

// Validation shared by the warp entry points; *s_out receives the cell size.
me_status check_warp(const char* who, const void* z_ref, void* z_out, int32_t dtype, int32_t C, int32_t Hf, int32_t Wf,
                     int32_t block, int32_t frame_h, int32_t frame_w, int* s_out)
{
    if (!z_ref || !z_out) return fail(ME_E_INVAL, "%s: null feature pointer", who);
    if (dtype != ME_F32 && dtype != ME_BF16) return fail(ME_E_INVAL, "%s: unknown dtype %d", who, dtype);
    if (C < 1 || Hf < 1 || Wf < 1) return fail(ME_E_INVAL, "%s: empty feature map", who);
    if ((long long)C * Hf * Wf > (1LL << 40)) return fail(ME_E_UNSUPPORTED, "%s: map too large", who);
    if ((long long)Hf * Wf > 0x7fffffffLL) return fail(ME_E_UNSUPPORTED, "%s: plane too large", who);
    if (!block_ok(block)) return fail(ME_E_UNSUPPORTED, "%s: block %d not in {8,16,32,64}", who, block);
    if (frame_h < 2 || frame_w < 2 || (frame_h & 1) || (frame_w & 1))
        return fail(ME_E_INVAL, "%s: frame size must be even and >= 2", who);
    const int Hp = frame_h / 2, Wp = frame_w / 2;
    if (Hp % Hf || Wp % Wf || Hp / Hf != Wp / Wf)
        return fail(ME_E_UNSUPPORTED, "%s: %dx%d map does not tile the %dx%d packed frame with square cells", who, Hf,
                    Wf, Hp, Wp);
    const int s = Hp / Hf;
    if (block % s) return fail(ME_E_UNSUPPORTED, "%s: cell size %d does not divide block %d", who, s, block);
    const size_t esz = dtype == ME_F32 ? 4 : 2;
    const char* a0 = static_cast<const char*>(z_ref);
    const char* b0 = static_cast<const char*>(z_out);
    const size_t bytes = (size_t)C * Hf * Wf * esz;
    if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(ME_E_INVAL, "%s: z_out overlaps z_ref", who);
    *s_out = s;
    return ME_OK;
}

}  // namespace

me_status me_warp_features(me_ctx ctx, const void* z_ref, void* z_out, int32_t dtype, int32_t C, int32_t Hf,
                           int32_t Wf, const int16_t* mv, int32_t block, int32_t frame_h, int32_t frame_w,
                           void* stream)
{
    (void)ctx;
    if (!mv) return fail(ME_E_INVAL, "me_warp_features: null pointer");
    int s = 0;
    me_status st = check_warp("me_warp_features", z_ref, z_out, dtype, C, Hf, Wf, block, frame_h, frame_w, &s);
    if (st != ME_OK) return st;
    if ((reinterpret_cast<uintptr_t>(mv) & 3u)) return fail(ME_E_INVAL, "me_warp_features: mv must be 4-byte aligned");
    const int bw = (frame_w / 2 + block - 1) / block;
    hipError_t e = launch_warp(z_ref, z_out, dtype == ME_BF16, C, Hf, Wf, mv, bw, block / s, s,
                               reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_warp_features: launch");
    return ME_OK;
}

me_status me_estimate_warp(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params* params, int16_t* mv,
                           int32_t* sad, const void* z_ref, void* z_out, int32_t dtype, int32_t C, int32_t Hf,
                           int32_t Wf, void* stream)
{
    me_status st = check_pair(ref, cur);
    if (st != ME_OK) return st;
    if (!params) return fail(ME_E_INVAL, "me_estimate_warp: null params");
    if (!mv || !sad) return fail(ME_E_INVAL, "me_estimate_warp: null mv or sad");
    const me_params& p = *params;
    if (!block_ok(p.block)) return fail(ME_E_UNSUPPORTED, "me_estimate_warp: block %d not in {8,16,32,64}", p.block);
    if (p.radius < 0 || p.radius > 64) return fail(ME_E_INVAL, "me_estimate_warp: radius %d not in [0,64]", p.radius);
    if (p.step != 1 || p.mode != ME_MODE_EXHAUSTIVE)
        return fail(ME_E_UNSUPPORTED, "me_estimate_warp: exhaustive mode with step 1 only");
    if ((reinterpret_cast<uintptr_t>(mv) & 3u)) return fail(ME_E_INVAL, "me_estimate_warp: mv must be 4-byte aligned");
    int s = 0;
    st = check_warp("me_estimate_warp", z_ref, z_out, dtype, C, Hf, Wf, p.block, cur->height, cur->width, &s);
    if (st != ME_OK) return st;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    SearchArgs a = make_args(ref, cur, p.block, p.radius, p.radius, nullptr, mv, sad);
    const TileCfg cfg = tiles_for(ctx, p.block, p.radius, a.Hp, a.Wp);
    hipError_t e;
    if (small_search(p.block, p.radius)) {
        // the small-radius kernel has no warp epilogue: search, then the warp kernel
        e = launch_sad_search(a, cfg, a.bh * a.bw, hs);
        if (e == hipSuccess)
            e = launch_warp(z_ref, z_out, dtype == ME_BF16, C, Hf, Wf, mv, a.bw, p.block / s, s, hs);
    } else {
        a.wz = z_ref;
        a.wout = z_out;
        a.wC = C;
        a.wHf = Hf;
        a.wWf = Wf;
        a.ws = s;
        a.wbf16 = dtype == ME_BF16;
        a.winv_s = 1.0f / (float)s;
        e = launch_sad_search(a, cfg, a.bh * a.bw, hs);
    }
    if (e != hipSuccess) return hip_fail(e, "me_estimate_warp: launch");
    return ME_OK;
}

me_status me_compose_vectors(const int16_t* mv_step, const int16_t* mv_acc_in, int16_t* mv_acc_out, int32_t block,
                             int32_t frame_h, int32_t frame_w, void* stream)
{
    if (!mv_step || !mv_acc_in || !mv_acc_out) return fail(ME_E_INVAL, "me_compose_vectors: null pointer");
    if (!block_ok(block)) return fail(ME_E_UNSUPPORTED, "me_compose_vectors: block %d not in {8,16,32,64}", block);
    if (frame_h < 2 || frame_w < 2 || (frame_h & 1) || (frame_w & 1) || frame_h > 65536 || frame_w > 65536)
        return fail(ME_E_INVAL, "me_compose_vectors: frame size must be even, 2..65536");
    const int Hp = frame_h / 2, Wp = frame_w / 2;
    const int bh = (Hp + block - 1) / block, bw = (Wp + block - 1) / block;
    const size_t bytes = (size_t)bh * bw * 2 * sizeof(int16_t);
    const char* o = reinterpret_cast<const char*>(mv_acc_out);
    const char* a = reinterpret_cast<const char*>(mv_acc_in);
    if (o < a + bytes && a < o + bytes) return fail(ME_E_INVAL, "me_compose_vectors: mv_acc_out overlaps mv_acc_in");
    hipError_t e = launch_compose(mv_step, mv_acc_in, mv_acc_out, bh, bw, block, Hp, Wp,
                                  reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_compose_vectors: launch");
    return ME_OK;
}

me_status me_refine(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params* params,
                    const float* net_out, int16_t* mv, int32_t* sad, uint8_t* fallback, void* stream)
{
    if (!ctx) return fail(ME_E_INVAL, "me_refine: null context");
    me_status s = check_pair(ref, cur);
    if (s != ME_OK) return s;
    if (!params || !net_out || !mv || !sad) return fail(ME_E_INVAL, "me_refine: null argument");
    s = check_refine_params(*params);
    if (s != ME_OK) return s;
    return refine_impl(ctx, ref, cur, *params, net_out, mv, sad, fallback, reinterpret_cast<hipStream_t>(stream));
}

me_status me_batch_submit(me_ctx ctx, const me_job* jobs, int32_t n, void* stream)
{
    if (!ctx) return fail(ME_E_INVAL, "me_batch_submit: null context");
    if (n < 0 || (n > 0 && !jobs)) return fail(ME_E_INVAL, "me_batch_submit: bad job array");
    for (int32_t k = 0; k < n; ++k) {
        const me_job& j = jobs[k];
        me_status s = check_pair(&j.ref, &j.cur);
        if (s != ME_OK) return s;
        if (!j.mv || !j.sad) return fail(ME_E_INVAL, "me_batch_submit: job %d: null mv or sad", k);
        if (!block_ok(j.params.block)) return fail(ME_E_UNSUPPORTED, "me_batch_submit: job %d: bad block", k);
        if (j.params.radius < 0 || j.params.radius > 64) return fail(ME_E_INVAL, "me_batch_submit: job %d: bad radius", k);
        if (j.params.step != 1 || j.params.mode != ME_MODE_EXHAUSTIVE)
            return fail(ME_E_UNSUPPORTED, "me_batch_submit: job %d: only exhaustive step-1 jobs", k);
    }
    if (n == 0) return ME_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);

    // shape of each job (block, radius, size, pitches): a submission whose
    // shapes repeat the previous one's replays the captured graph
    std::vector<int64_t> shapes((size_t)n * 4);
    for (int32_t k = 0; k < n; ++k) {
        const me_job& j = jobs[k];
        shapes[4 * k] = (int64_t)j.params.block << 32 | (uint32_t)j.params.radius;
        shapes[4 * k + 1] = (int64_t)j.cur.height << 32 | (uint32_t)j.cur.width;
        shapes[4 * k + 2] = j.ref.pitch;
        shapes[4 * k + 3] = j.cur.pitch;
    }
    const bool same = ctx->graph && shapes == ctx->batch_shapes;

    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (!ctx->staged) {
        if ((e = hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming)) != hipSuccess ||
            (e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "me_batch_submit: setup");
    }
    if (!ctx->qcount) {
        if (hipMalloc(&ctx->qcount, sizeof(int32_t) * kQueueCounters) != hipSuccess)
            return fail(ME_E_NOMEM, "me_batch_submit: queue counters");
        if ((e = launch_fill_i32(ctx->qcount, kQueueCounters, 0, st)) != hipSuccess)
            return hip_fail(e, "me_batch_submit: queue counters");
    }

    // plan (new shapes only):
    //  * full-width blocks: one persistent queue launch per block size over
    //    all its jobs, jobs in decreasing order of work per item;
    //  * blocks cut by the right frame edge: per-shape launches of the generic
    //    kernel over a (job, block row) grid, pointers from a shape-grouped table.
    std::vector<int32_t> slot((size_t)n);
    std::vector<std::pair<int32_t, int32_t>> groups;     // partial-width shape groups: (first job, count)
    std::vector<QueueJob> qplan;
    std::vector<int32_t> qrow_job;
    std::vector<QueueLaunch> qlaunch;
    if (same) {
        slot = ctx->batch_slot;
    } else {
        std::vector<std::vector<int32_t>> members;
        std::map<std::vector<int64_t>, size_t> index;
        for (int32_t k = 0; k < n; ++k) {
            std::vector<int64_t> key(shapes.begin() + 4 * k, shapes.begin() + 4 * k + 4);
            auto it = index.find(key);
            if (it == index.end()) {
                it = index.emplace(key, members.size()).first;
                members.emplace_back();
            }
            members[it->second].push_back(k);
        }
        int32_t row = 0;
        for (const std::vector<int32_t>& m : members) {
            groups.push_back({m[0], (int32_t)m.size()});
            for (int32_t k : m) slot[k] = row++;
        }
        for (int B : {8, 16, 32, 64}) {
            std::vector<int32_t> ks;
            for (int32_t k = 0; k < n; ++k) {
                const me_job& j = jobs[k];
                if (j.params.block == B && (j.cur.width / 2) / B > 0) ks.push_back(k);
            }
            if (ks.empty()) continue;
            // tile shape of the queue kernel: 4x2 tiles, remainder rows as single
            // candidates, current block through scalar loads (its register count
            // keeps four waves per SIMD); per-pair tunings do not carry over, since
            // the queue kernel's registers differ from the single-pair kernel's
            TileCfg tile{};
            tile.kx = 4;
            tile.ky = 2;
            tile.rs = 1;
            QueueLaunch ql{};
            ql.block = B;
            ql.tile = tile;
            ql.first = (int32_t)qplan.size();
            std::vector<std::pair<double, int32_t>> order;   // (-work per item, job)
            std::vector<QueueJob> plans((size_t)n);
            for (int32_t k : ks) {
                const me_job& j = jobs[k];
                QueueJob& q = plans[k];
                q = QueueJob{};
                q.ref_pitch = j.ref.pitch / 2;
                q.cur_pitch = j.cur.pitch / 2;
                q.Hp = j.cur.height / 2;
                q.Wp = j.cur.width / 2;
                q.bh = (q.Hp + B - 1) / B;
                q.bw = (q.Wp + B - 1) / B;
                q.R = j.params.radius;
                size_t bytes = 0;
                if (!plan_queue_job(B, tile, kLdsQueue, &q, &bytes) && !plan_queue_job(B, tile, kLdsQueueMax, &q, &bytes))
                    return fail(ME_E_UNSUPPORTED, "me_batch_submit: job %d: no window plan for block %d radius %d", k,
                                B, q.R);
                if (bytes > ql.lds_bytes) ql.lds_bytes = bytes;
                const double nc = 2.0 * q.R + 1.0;
                order.push_back({-(double)q.nb * nc * nc, k});
            }
            std::stable_sort(order.begin(), order.end(),
                             [](const std::pair<double, int32_t>& a, const std::pair<double, int32_t>& b) {
                                 return a.first < b.first;
                             });
            int64_t items = 0;
            for (const auto& o : order) {
                QueueJob q = plans[o.second];
                q.item0 = (int32_t)items;
                items += (int64_t)q.bh * q.groups;
                if (items > 0x7fffffff) return fail(ME_E_UNSUPPORTED, "me_batch_submit: too many blocks");
                qplan.push_back(q);
                qrow_job.push_back(o.second);
            }
            ql.n_jobs = (int32_t)qplan.size() - ql.first;
            ql.n_items = (int32_t)items;
            ql.counter = (int32_t)qlaunch.size();
            if (ql.counter >= kQueueCounters) return fail(ME_E_UNSUPPORTED, "me_batch_submit: too many block sizes");
            qlaunch.push_back(ql);
        }
    }

    // the previous submission's staging copies must be done before reuse
    if ((e = hipEventSynchronize(ctx->staged)) != hipSuccess) return hip_fail(e, "me_batch_submit: staging wait");
    const size_t nq = same ? ctx->qplan.size() : qplan.size();
    if ((size_t)n > ctx->cap_ptrs || nq > ctx->cap_q) {
        // larger tables move: wait for launches that may still read the old
        // ones, and drop the graph that captured their addresses
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "me_batch_submit: synchronize");
        if (ctx->graph) {
            (void)hipGraphExecDestroy(ctx->graph);
            ctx->graph = nullptr;
        }
        ctx->batch_shapes.clear();
        if ((size_t)n > ctx->cap_ptrs) {
            (void)hipFree(ctx->ptrs_dev);
            (void)hipHostFree(ctx->ptrs_host);
            ctx->ptrs_dev = nullptr;
            ctx->ptrs_host = nullptr;
            ctx->cap_ptrs = 0;
            if (hipMalloc(&ctx->ptrs_dev, sizeof(JobPtrs) * n) != hipSuccess ||
                hipHostMalloc(&ctx->ptrs_host, sizeof(JobPtrs) * n) != hipSuccess)
                return fail(ME_E_NOMEM, "me_batch_submit: pointer table allocation failed");
            ctx->cap_ptrs = (size_t)n;
        }
        if (nq > ctx->cap_q) {
            (void)hipFree(ctx->qjobs_dev);
            (void)hipHostFree(ctx->qjobs_host);
            ctx->qjobs_dev = nullptr;
            ctx->qjobs_host = nullptr;
            ctx->cap_q = 0;
            if (hipMalloc(&ctx->qjobs_dev, sizeof(QueueJob) * nq) != hipSuccess ||
                hipHostMalloc(&ctx->qjobs_host, sizeof(QueueJob) * nq) != hipSuccess)
                return fail(ME_E_NOMEM, "me_batch_submit: queue table allocation failed");
            ctx->cap_q = nq;
        }
    }
    if (!same) {
        // a new plan: its tables are staged below and its launches captured
        if (ctx->graph) {
            (void)hipGraphExecDestroy(ctx->graph);
            ctx->graph = nullptr;
        }
        ctx->batch_shapes.clear();
        ctx->qplan.swap(qplan);
        ctx->qrow_job.swap(qrow_job);
        ctx->qlaunch.swap(qlaunch);
    }
    for (int32_t k = 0; k < n; ++k) {
        const me_job& j = jobs[k];
        JobPtrs& p = ctx->ptrs_host[slot[k]];
        p.ref = reinterpret_cast<const uint32_t*>(j.ref.data);
        p.cur = reinterpret_cast<const uint32_t*>(j.cur.data);
        p.mv = j.mv;
        p.sad = j.sad;
    }
    for (size_t r = 0; r < nq; ++r) {
        const me_job& j = jobs[ctx->qrow_job[r]];
        QueueJob q = ctx->qplan[r];
        q.ref = reinterpret_cast<const uint32_t*>(j.ref.data);
        q.cur = reinterpret_cast<const uint32_t*>(j.cur.data);
        q.mv = j.mv;
        q.sad = j.sad;
        ctx->qjobs_host[r] = q;
    }
    if ((e = hipMemcpyAsync(ctx->ptrs_dev, ctx->ptrs_host, sizeof(JobPtrs) * n, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (nq > 0 && (e = hipMemcpyAsync(ctx->qjobs_dev, ctx->qjobs_host, sizeof(QueueJob) * nq,
                                       hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (e = hipEventRecord(ctx->staged, st)) != hipSuccess)
        return hip_fail(e, "me_batch_submit: staging copy");

    // one captured graph of the queue launches and the generic launches; they
    // read the tables at fixed addresses, so a replay picks up new pairs
    if (!same) {
        std::vector<SearchArgs> args;
        std::vector<TileCfg> cfgs;
        for (const std::pair<int32_t, int32_t>& g : groups) {
            const me_job& j = jobs[g.first];
            if ((j.cur.width / 2) % j.params.block == 0) continue;      // no block cut by the right edge
            SearchArgs a = make_args(&j.ref, &j.cur, j.params.block, j.params.radius, j.params.radius, nullptr,
                                     j.mv, j.sad);
            a.jobs = ctx->ptrs_dev + slot[g.first];
            a.n_jobs = g.second;
            args.push_back(a);
            cfgs.push_back(tiles_for(ctx, a.block, a.R, a.Hp, a.Wp));
        }
        hipGraph_t gr = nullptr;
        if ((e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "me_batch_submit: capture");
        hipError_t le = hipSuccess;
        for (size_t i = 0; i < ctx->qlaunch.size() && le == hipSuccess; ++i) {
            const QueueLaunch& ql = ctx->qlaunch[i];
            QueueArgs q{};
            q.jobs = ctx->qjobs_dev + ql.first;
            q.n_jobs = ql.n_jobs;
            q.n_items = ql.n_items;
            q.counter = ctx->qcount + ql.counter;
            le = launch_sad_queue(q, ql.block, ql.tile, ql.lds_bytes, ctx->capture_stream);
        }
        for (size_t i = 0; i < args.size() && le == hipSuccess; ++i)
            le = launch_sad_search(args[i], cfgs[i], 0, ctx->capture_stream, 2);
        e = hipStreamEndCapture(ctx->capture_stream, &gr);
        if (le != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return hip_fail(le, "me_batch_submit: captured launch");
        }
        if (e != hipSuccess) return hip_fail(e, "me_batch_submit: end capture");
        e = hipGraphInstantiate(&ctx->graph, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return hip_fail(e, "me_batch_submit: instantiate");
        ctx->batch_shapes.swap(shapes);
        ctx->batch_slot.swap(slot);
    }
    if ((e = hipGraphLaunch(ctx->graph, st)) != hipSuccess) return hip_fail(e, "me_batch_submit: graph launch");
    return ME_OK;
}

me_status me_sync(void* stream)
{
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_sync: work on the stream failed");
    return ME_OK;
}

namespace {

me_status check_sad_maps(const char* who, const int32_t* sad, int32_t n, int32_t block, int32_t frame_h,
                         int32_t frame_w, int* bh, int* bw)
{
    if (!sad) return fail(ME_E_INVAL, "%s: null sad", who);
    if (n < 1) return fail(ME_E_INVAL, "%s: n = %d, need at least one map", who, n);
    if (!block_ok(block)) return fail(ME_E_UNSUPPORTED, "%s: block %d not in {8,16,32,64}", who, block);
    if (frame_h < 2 || frame_w < 2 || (frame_h & 1) || (frame_w & 1) || frame_h > 65536 || frame_w > 65536)
        return fail(ME_E_INVAL, "%s: frame size must be even, 2..65536", who);
    *bh = (frame_h / 2 + block - 1) / block;
    *bw = (frame_w / 2 + block - 1) / block;
    return ME_OK;
}

}  // namespace

me_status me_sad_median(me_ctx ctx, const int32_t* sad, int32_t n, int32_t block, int32_t frame_h, int32_t frame_w,
                        float* median, void* stream)
{
    if (!ctx || !median) return fail(ME_E_INVAL, "me_sad_median: null context or output");
    int bh = 0, bw = 0;
    me_status s = check_sad_maps("me_sad_median", sad, n, block, frame_h, frame_w, &bh, &bw);
    if (s != ME_OK) return s;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (!ctx->stat && hipMalloc(&ctx->stat, 260 * sizeof(uint32_t)) != hipSuccess)
        return fail(ME_E_NOMEM, "me_sad_median: scratch allocation failed");
    const int64_t N = (int64_t)n * bh * bw;
    e = launch_sad_median(sad, N, bh * bw, bw, frame_h / 2, frame_w / 2, block, ctx->stat, ctx->stat + 256, median,
                          reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_sad_median: launch");
    return ME_OK;
}

me_status me_fallback_weight(const int32_t* sad, int32_t n, int32_t block, int32_t frame_h, int32_t frame_w,
                             float sad_ratio, float median_per_sample, float* weight, void* stream)
{
    if (!weight) return fail(ME_E_INVAL, "me_fallback_weight: null weight");
    int bh = 0, bw = 0;
    me_status s = check_sad_maps("me_fallback_weight", sad, n, block, frame_h, frame_w, &bh, &bw);
    if (s != ME_OK) return s;
    if (!(sad_ratio >= 0.0f) || !(median_per_sample >= 0.0f))
        return fail(ME_E_INVAL, "me_fallback_weight: ratio and median must be >= 0");
    const double ratio_m = (double)sad_ratio * (double)median_per_sample;
    hipError_t e = launch_fallback_weight(sad, (int64_t)n * bh * bw, bh * bw, bw, frame_h / 2, frame_w / 2, block,
                                          ratio_m, weight, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "me_fallback_weight: launch");
    return ME_OK;
}

// Records `c` as the launch shape for (block, radius, Hp, Wp).  A captured batch
// graph holds the shapes it was recorded with: it is dropped, so the next
// submission records the new one.
static me_status store_shape(me_ctx ctx, int block, int radius, int Hp, int Wp, const TileCfg& c, const char* who)
{
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->tuned[std::make_tuple(block, radius, Hp, Wp)] = c;
    }
    if (ctx->graph) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, who);
        (void)hipGraphExecDestroy(ctx->graph);
        ctx->graph = nullptr;
    }
    ctx->batch_shapes.clear();
    return ME_OK;
}

me_status me_autotune(me_ctx ctx, const me_frame* ref, const me_frame* cur, int32_t block, int32_t radius,
                      int32_t iters, float* best_ms, void* stream)
{
    if (!ctx) return fail(ME_E_INVAL, "me_autotune: null context");
    me_status s = check_pair(ref, cur);
    if (s != ME_OK) return s;
    if (!block_ok(block)) return fail(ME_E_UNSUPPORTED, "me_autotune: block %d not in {8,16,32,64}", block);
    if (radius < 0 || radius > 64) return fail(ME_E_INVAL, "me_autotune: radius %d not in [0,64]", radius);
    if (iters < 1 || iters > 100) return fail(ME_E_INVAL, "me_autotune: iters %d not in [1,100]", iters);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int Hp = cur->height / 2, Wp = cur->width / 2;
    const size_t nblk = (size_t)((Hp + block - 1) / block) * ((Wp + block - 1) / block);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (nblk > ctx->tune_cap) {
        (void)hipFree(ctx->tune_mv);
        (void)hipFree(ctx->tune_sad);
        ctx->tune_mv = nullptr;
        ctx->tune_sad = nullptr;
        ctx->tune_cap = 0;
        if (hipMalloc(&ctx->tune_mv, nblk * 2 * sizeof(int16_t)) != hipSuccess ||
            hipMalloc(&ctx->tune_sad, nblk * sizeof(int32_t)) != hipSuccess)
            return fail(ME_E_NOMEM, "me_autotune: allocation failed");
        ctx->tune_cap = nblk;
    }
    SearchArgs a = make_args(ref, cur, block, radius, radius, nullptr, ctx->tune_mv, ctx->tune_sad);
    const int shapes[6][2] = {{4, 4}, {8, 2}, {4, 2}, {8, 4}, {8, 1}, {4, 1}};
    const size_t caps[3] = {53 * 1024, 80 * 1024, 158 * 1024};
    std::vector<TileCfg> cands;
    const int groupings[4][2] = {{1, 4}, {2, 4}, {2, 2}, {4, 2}};   // (blocks, waves per block)
    for (auto& sh : shapes)
        for (auto& gp : groupings)
            for (int cl : {0, 1}) {
                const int nb = gp[0];
                if (nb > 1 && radius % 4) continue;
                for (size_t cap : caps) {
                    TileCfg c{};
                    c.kx = sh[0];
                    c.ky = sh[1];
                    c.nb = nb;
                    c.wpb = gp[1];
                    c.cl = cl;
                    c.rs = 1;
                    if (!tiles_supported(block, c.kx, c.ky) || !plan_tiles(block, radius, cap, &c)) continue;
                    bool dup = false;
                    for (const TileCfg& o : cands)
                        dup |= o.kx == c.kx && o.ky == c.ky && o.nb == c.nb && o.band_ty == c.band_ty &&
                               o.lds_pitch == c.lds_pitch && o.cl == c.cl && o.wpb == c.wpb;
                    if (!dup) cands.push_back(c);
                }
            }
    hipEvent_t t0, t1;
    if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess)
        return hip_fail(e, "me_autotune: events");
    float best = 1e30f;
    TileCfg best_cfg = default_tiles(block, radius);
    for (const TileCfg& c : cands) {
        e = launch_sad_search(a, c, 0, st);               // warm-up (and launch check)
        if (e != hipSuccess) continue;
        (void)hipEventRecord(t0, st);
        for (int i = 0; i < iters; ++i) (void)launch_sad_search(a, c, 0, st);
        (void)hipEventRecord(t1, st);
        if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        ms /= (float)iters;
        if (ms < best) {
            best = ms;
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e, "me_autotune: timing");
    if ((s = store_shape(ctx, block, radius, Hp, Wp, best_cfg, "me_autotune")) != ME_OK) return s;
    if (best_ms) *best_ms = best;
    return ME_OK;
}

me_status me_tuned_shape(me_ctx ctx, int32_t block, int32_t radius, int32_t height, int32_t width, int32_t* shape,
                         int32_t* tuned)
{
    if (!ctx || !shape) return fail(ME_E_INVAL, "me_tuned_shape: null context or shape");
    if (!block_ok(block)) return fail(ME_E_UNSUPPORTED, "me_tuned_shape: block %d not in {8,16,32,64}", block);
    if (radius < 0 || radius > 64) return fail(ME_E_INVAL, "me_tuned_shape: radius %d not in [0,64]", radius);
    if (height < 2 || width < 2 || (height & 1) || (width & 1))
        return fail(ME_E_INVAL, "me_tuned_shape: frame %dx%d not even and positive", height, width);
    const int Hp = height / 2, Wp = width / 2;
    bool found = false;
    TileCfg c{};
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->tuned.find(std::make_tuple(block, radius, Hp, Wp));
        if (it != ctx->tuned.end()) {
            c = it->second;
            found = true;
        }
    }
    if (!found) c = default_tiles(block, radius);
    shape[0] = c.kx;
    shape[1] = c.ky;
    shape[2] = c.nb;
    shape[3] = (int32_t)((c.lds_bytes + 1023) / 1024);
    shape[4] = c.cl;
    shape[5] = c.wpb ? c.wpb : 4;
    if (tuned) *tuned = found ? 1 : 0;
    return ME_OK;
}

me_status me_set_tuned_shape(me_ctx ctx, int32_t block, int32_t radius, int32_t height, int32_t width,
                             const int32_t* shape)
{
    if (!ctx || !shape) return fail(ME_E_INVAL, "me_set_tuned_shape: null context or shape");
    if (!block_ok(block)) return fail(ME_E_UNSUPPORTED, "me_set_tuned_shape: block %d not in {8,16,32,64}", block);
    if (radius < 0 || radius > 64) return fail(ME_E_INVAL, "me_set_tuned_shape: radius %d not in [0,64]", radius);
    if (height < 2 || width < 2 || (height & 1) || (width & 1))
        return fail(ME_E_INVAL, "me_set_tuned_shape: frame %dx%d not even and positive", height, width);
    TileCfg c{};
    c.kx = shape[0];
    c.ky = shape[1];
    c.nb = shape[2];
    c.cl = shape[4];
    c.wpb = shape[5];
    c.rs = 1;
    if (c.cl != 0 && c.cl != 1)
        return fail(ME_E_INVAL, "me_set_tuned_shape: current-block source %d not 0 or 1", c.cl);
    if (c.wpb != 2 && c.wpb != 4 && c.wpb != 8)
        return fail(ME_E_INVAL, "me_set_tuned_shape: %d waves per block (2, 4 or 8)", c.wpb);
    if (!tiles_supported(block, c.kx, c.ky))
        return fail(ME_E_UNSUPPORTED, "me_set_tuned_shape: tile %dx%d not compiled for block %d", c.kx, c.ky, block);
    if (c.nb < 1 || c.nb * c.wpb > 8 || (c.nb > 1 && radius % 4))
        return fail(ME_E_UNSUPPORTED,
                    "me_set_tuned_shape: %d blocks of %d waves per workgroup (at most 8 waves; one block unless "
                    "radius %% 4 == 0)", c.nb, c.wpb);
    if (shape[3] < 1 || shape[3] > 158 || !plan_tiles(block, radius, (size_t)shape[3] * 1024, &c))
        return fail(ME_E_UNSUPPORTED, "me_set_tuned_shape: no window band fits in %d KB of LDS (at most 158)",
                    shape[3]);
    return store_shape(ctx, block, radius, height / 2, width / 2, c, "me_set_tuned_shape");
}

}  // extern "C"
