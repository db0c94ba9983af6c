// me_refine_noalloc: the refine-and-fallback step with its scratch (decoded
// proposals, fallback flags, the compacted fallback list and its count) in a
// fixed device array of the library instead of buffers the context grows
// with hipMalloc.  Same kernels and launch sequence as me_refine.
#include "ctx.h"

namespace me {
namespace {

constexpr size_t kBlocks = ME_NOALLOC_MAX_BLOCKS;
constexpr size_t kOffPred = 0;                       // int16 [kBlocks][2]
constexpr size_t kOffList = 4 * kBlocks;              // int32 [kBlocks]
constexpr size_t kOffFb = 8 * kBlocks;                // uint8 [kBlocks]
constexpr size_t kOffCount = 9 * kBlocks;             // int32, own 256-byte line
constexpr size_t kBytes = kOffCount + 256;
static_assert(kOffCount % 256 == 0, "count slot must start a 256-byte line");

// One copy per device, alive until the process ends.  Host code never passes
// this name to a kernel: it takes the per-device address resolved below.
static __device__ __align__(256) unsigned char scratch[kBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on `device`, resolved once per device with that
// device current (the caller's current device is restored).
me_status noalloc_resolve(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(ME_E_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr[device]) return ME_OK;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) {
        const hipError_t r = hipSetDevice(prev);
        if (e == hipSuccess && r != hipSuccess) return hip_fail(r, "hipSetDevice (restore)");
    }
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(ME_E_HIP, "hipGetSymbolAddress(scratch) returned null");
    g_ptr[device] = static_cast<unsigned char*>(p);
    return ME_OK;
}

}  // namespace me

extern "C" me_status me_refine_noalloc(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params* params,
                                       const float* net_out, int16_t* mv, int32_t* sad, uint8_t* fallback,
                                       void* stream)
{
    using namespace me;
    me_status s = check_pair(ref, cur);
    if (s != ME_OK) return s;
    if (!params || !net_out || !mv || !sad) return fail(ME_E_INVAL, "me_refine_noalloc: null argument");
    s = check_refine_params(*params);
    if (s != ME_OK) return s;
    const me_params& p = *params;
    const int Hp = cur->height / 2, Wp = cur->width / 2;
    const int64_t bh = (Hp + p.block - 1) / p.block, bw = (Wp + p.block - 1) / p.block;
    if (bh * bw > (int64_t)kBlocks)
        return fail(ME_E_INVAL, "me_refine_noalloc: %lld blocks exceed the fixed scratch of %d blocks",
                    (long long)(bh * bw), ME_NOALLOC_MAX_BLOCKS);
    if (!ctx) return fail(ME_E_INVAL, "me_refine_noalloc: null context");
    const float m = p.sad_median_per_sample > 0.0f ? p.sad_median_per_sample : ctx->median_per_sample;
    if (!(m > 0.0f)) return fail(ME_E_STATE, "me_refine_noalloc: no SAD median (params or loaded weights)");
    unsigned char* base;
    {
        std::lock_guard<std::mutex> g(g_mu);
        base = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_ptr[ctx->device] : nullptr;
    }
    if (!base) return fail(ME_E_STATE, "me_refine_noalloc: scratch of device %d not resolved", ctx->device);
    const RefineScratch w{reinterpret_cast<int16_t*>(base + kOffPred), base + kOffFb,
                          reinterpret_cast<int32_t*>(base + kOffList), reinterpret_cast<int32_t*>(base + kOffCount)};
    return refine_run(ref, cur, p, m, net_out, mv, sad, fallback, w, reinterpret_cast<hipStream_t>(stream));
}
