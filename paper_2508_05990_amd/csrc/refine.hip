// Learned-proposal mode, refine and fallback: the network's per-block output
// (mvx, mvy in units of 8 packed pixels, confidence logit) is decoded into an
// integer proposal, an exact small-radius stage search runs around it (the
// same kernel as full search, with per-block predictors), and blocks whose
// proposal is not trusted are compacted into a device list that the full
// search then processes -- no host round trip between the steps.
#include "internal.h"

namespace me {
namespace {

// p = clamp(rint(8 o), -R, R) for both components, rounding half to even.
__global__ void decode_kernel(const float* __restrict__ out, int nblk, int R, int16_t* __restrict__ pred)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const float px = rintf(8.0f * out[b]);
    const float py = rintf(8.0f * out[nblk + b]);
    const float r = (float)R;
    pred[2 * b] = (int16_t)fminf(fmaxf(px, -r), r);
    pred[2 * b + 1] = (int16_t)fminf(fmaxf(py, -r), r);
}

// Fallback test per block, then an ordered compaction of the fallback blocks
// into list[0 .. *count).  One workgroup; blocks are visited in chunks of
// blockDim.x, each chunk compacted with a wave ballot and a workgroup prefix.
__global__ __launch_bounds__(1024) void fallback_kernel(const float* __restrict__ out, const int32_t* __restrict__ sad,
                                                        int nblk, int bh, int bw, int Hp, int Wp, int B,
                                                        float conf_thresh, double ratio_m, uint8_t* __restrict__ fb,
                                                        int32_t* __restrict__ list, int32_t* __restrict__ count)
{
    __shared__ int wave_base[16];
    __shared__ int total;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    if (tid == 0) total = 0;
    __syncthreads();
    const float* logit = out + 2 * nblk;
    for (int c0 = 0; c0 < nblk; c0 += blockDim.x) {
        const int b = c0 + tid;
        bool f = false;
        if (b < nblk) {
            const int bi = b / bw, bj = b - bi * bw;
            const int h = min(B, Hp - bi * B), w = min(B, Wp - bj * B);
            const double n = 4.0 * h * w;
            const long long thr = (long long)floor(ratio_m * n);
            const int s = sad[b];
            f = (logit[b] < conf_thresh) || s < 0 || (long long)s > thr;
            fb[b] = f ? 1 : 0;
        }
        const unsigned long long m = __ballot(f);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wave_base[wave] = __popcll(m);
        __syncthreads();
        if (tid == 0) {
            int run = total;
            for (int k = 0; k < nw; ++k) {
                const int c = wave_base[k];
                wave_base[k] = run;
                run += c;
            }
            total = run;
        }
        __syncthreads();
        if (f) list[wave_base[wave] + before] = b;
        __syncthreads();
    }
    if (tid == 0) *count = total;
}

}  // namespace

hipError_t launch_decode(const float* out, int nblk, int R, int16_t* pred, hipStream_t stream)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(decode_kernel, dim3((nblk + 255) / 256), dim3(256), 0, stream, out, nblk, R, pred);
    return hipGetLastError();
}

hipError_t launch_fallback(const float* out, const int32_t* sad, int bh, int bw, int Hp, int Wp, int B,
                           float conf_thresh, double ratio_m, uint8_t* fb, int32_t* list, int32_t* count,
                           hipStream_t stream)
{
    hipLaunchKernelGGL(fallback_kernel, dim3(1), dim3(1024), 0, stream, out, sad, bh * bw, bh, bw, Hp, Wp, B,
                       conf_thresh, ratio_m, fb, list, count);
    return hipGetLastError();
}

}  // namespace me
