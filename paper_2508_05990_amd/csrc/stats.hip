// Training-set statistics of the learned-proposal mode, on the GPU: the
// median per-sample full-search SAD (the M of the SAD fallback test) and the
// per-block weight of the vector term (0 where the full-search match is too
// poor for any proposal to be accepted).
//
// Per-sample SAD of block b of map k: q = fl32(fl32(sad) / fl32(n_b)), n_b =
// 4 h w the block's sample count.  The median is the lower median, the
// element of rank floor((N - 1) / 2) in ascending order, found by a four-pass
// radix select over an order-preserving 32-bit key of q: each pass counts the
// keys that share the prefix chosen so far by their next byte, and one
// workgroup picks the byte whose bin holds the wanted rank.  Counts are exact
// integers, so the result does not depend on the order of the atomics.
#include "internal.h"

namespace me {
namespace {

__device__ __forceinline__ float per_sample(int32_t s, int blk, int bw, int Hp, int Wp, int B)
{
    const int bi = blk / bw, bj = blk - bi * bw;
    const int h = min(B, Hp - bi * B), w = min(B, Wp - bj * B);
    return (float)s / (float)(4 * h * w);
}

// Order-preserving key: ascending floats give ascending unsigned keys.
__device__ __forceinline__ uint32_t fkey(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float fkey_inv(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// state[0] = chosen prefix, state[1] = rank still wanted within it.
__global__ void select_init_kernel(uint32_t* __restrict__ hist, uint32_t* __restrict__ state, uint32_t rank)
{
    hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        state[0] = 0u;
        state[1] = rank;
    }
}

__global__ __launch_bounds__(256) void select_hist_kernel(const int32_t* __restrict__ sad, int64_t N, int nblk, int bw,
                                                          int Hp, int Wp, int B, int pass,
                                                          const uint32_t* __restrict__ state,
                                                          uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t prefix = state[0];
    const int shift = 24 - 8 * pass;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
        const int blk = (int)(e % nblk);
        const uint32_t k = fkey(per_sample(sad[e], blk, bw, Hp, Wp, B));
        if (pass == 0 || (k >> (shift + 8)) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Picks the byte of this pass, clears the histogram for the next pass; after
// the last pass writes the median.
__global__ void select_pick_kernel(uint32_t* __restrict__ hist, uint32_t* __restrict__ state, int pass,
                                   float* __restrict__ median)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = hist[threadIdx.x];
    hist[threadIdx.x] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t r = state[1], before = 0u, b = 0u;
        for (; b < 255u; ++b) {
            if (before + cnt[b] > r) break;
            before += cnt[b];
        }
        const uint32_t prefix = (state[0] << 8) | b;
        state[0] = prefix;
        state[1] = r - before;
        if (pass == 3) *median = fkey_inv(prefix);
    }
}

// weight = 1 where sad <= floor(ratio_m * n_b) (product in double, the SAD
// fallback threshold), else 0.
__global__ void weight_kernel(const int32_t* __restrict__ sad, int64_t N, int nblk, int bw, int Hp, int Wp, int B,
                              double ratio_m, float* __restrict__ weight)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const int blk = (int)(e % nblk);
    const int bi = blk / bw, bj = blk - bi * bw;
    const int h = min(B, Hp - bi * B), w = min(B, Wp - bj * B);
    const long long thr = (long long)floor(ratio_m * (4.0 * h * w));
    weight[e] = (long long)sad[e] <= thr ? 1.0f : 0.0f;
}

}  // namespace

hipError_t launch_sad_median(const int32_t* sad, int64_t N, int nblk, int bw, int Hp, int Wp, int B, uint32_t* hist,
                             uint32_t* state, float* median, hipStream_t st)
{
    hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, st, hist, state, (uint32_t)((N - 1) / 2));
    int64_t wg = (N + 255) / 256;
    if (wg > 2048) wg = 2048;
    for (int pass = 0; pass < 4; ++pass) {
        hipLaunchKernelGGL(select_hist_kernel, dim3((unsigned)wg), dim3(256), 0, st, sad, N, nblk, bw, Hp, Wp, B, pass,
                           state, hist);
        hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(256), 0, st, hist, state, pass, median);
    }
    return hipGetLastError();
}

hipError_t launch_fallback_weight(const int32_t* sad, int64_t N, int nblk, int bw, int Hp, int Wp, int B,
                                  double ratio_m, float* weight, hipStream_t st)
{
    const int64_t wg = (N + 255) / 256;
    if (wg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(weight_kernel, dim3((unsigned)wg), dim3(256), 0, st, sad, N, nblk, bw, Hp, Wp, B, ratio_m,
                       weight);
    return hipGetLastError();
}

}  // namespace me
