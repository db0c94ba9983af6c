// Propagation of a reference feature map by per-block motion vectors,
// z_pred = Warp(z_R, MV) (paper Sec. 3.3), on gfx950.
//
// HBM-bound: every output element reads four neighbouring inputs (mostly
// L2/L1 hits, since neighbouring cells of a block share one vector) and is
// written once.  The vector, the clamped row and column indices and the four
// bilinear weights are computed once per thread and reused for every channel
// of its chunk; consecutive lanes take consecutive cells of a row, so loads
// and stores of a channel plane are contiguous across the wave.
#include "internal.h"

namespace me {
namespace {

__device__ __forceinline__ float bf16_to_f32(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

// Round to nearest, ties to even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ int floor_div(int a, int b)
{
    const int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

template <bool BF16>
__global__ __launch_bounds__(256) void warp_kernel(const void* __restrict__ zin, void* __restrict__ zout, int C,
                                                   int Hf, int Wf, const int16_t* __restrict__ mv, int bw, int cells,
                                                   int s, float inv_s, int cpt)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncell = Hf * Wf;
    if (cell >= ncell) return;
    const int i = cell / Wf, j = cell - i * Wf;
    const int c0 = blockIdx.y * cpt;
    const int c1 = min(C, c0 + cpt);

    const int b = (i / cells) * bw + (j / cells);
    const int32_t vec = reinterpret_cast<const int32_t*>(mv)[b];   // (dx, dy) as two int16
    const int dx = (int16_t)(vec & 0xffff), dy = (int16_t)((uint32_t)vec >> 16);
    const int ny = i * s + dy, nx = j * s + dx;
    const int y0 = floor_div(ny, s), x0 = floor_div(nx, s);
    const float wy = (float)(ny - y0 * s) * inv_s;
    const float wx = (float)(nx - x0 * s) * inv_s;
    const int ya = min(max(y0, 0), Hf - 1), yb = min(max(y0 + 1, 0), Hf - 1);
    const int xa = min(max(x0, 0), Wf - 1), xb = min(max(x0 + 1, 0), Wf - 1);
    const float w00 = (1.f - wy) * (1.f - wx), w01 = (1.f - wy) * wx;
    const float w10 = wy * (1.f - wx), w11 = wy * wx;
    const int o00 = ya * Wf + xa, o01 = ya * Wf + xb, o10 = yb * Wf + xa, o11 = yb * Wf + xb;

    const size_t plane = (size_t)ncell;
    for (int c = c0; c < c1; ++c) {
        const size_t base = (size_t)c * plane;
        float v00, v01, v10, v11;
        if (BF16) {
            const uint16_t* p = reinterpret_cast<const uint16_t*>(zin) + base;
            v00 = bf16_to_f32(p[o00]);
            v01 = bf16_to_f32(p[o01]);
            v10 = bf16_to_f32(p[o10]);
            v11 = bf16_to_f32(p[o11]);
        } else {
            const float* p = reinterpret_cast<const float*>(zin) + base;
            v00 = p[o00];
            v01 = p[o01];
            v10 = p[o10];
            v11 = p[o11];
        }
        float acc = w00 * v00;
        acc = fmaf(w01, v01, acc);
        acc = fmaf(w10, v10, acc);
        acc = fmaf(w11, v11, acc);
        if (BF16)
            reinterpret_cast<uint16_t*>(zout)[base + cell] = f32_to_bf16(acc);
        else
            reinterpret_cast<float*>(zout)[base + cell] = acc;
    }
}

// Runs of four horizontally adjacent cells inside one block (cells per block
// a multiple of 4): the run shares one vector, so its four outputs read five
// consecutive inputs from each of two rows and are written as one vector.
// Each thread owns one run and a chunk of channels, four channels in flight.
template <bool BF16>
__global__ __launch_bounds__(256) void warp_run_kernel(const void* __restrict__ zin, void* __restrict__ zout, int C,
                                                       int Hf, int Wf, const int16_t* __restrict__ mv, int bw,
                                                       int cells, int s, float inv_s, int cpt, int runs_per_row,
                                                       int n_runs)
{
    // work item = (channel chunk, run); XCD-contiguous ranges of items
    const int nwg = gridDim.x;
    const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
    const int q = nwg >> 3, rem = nwg & 7;
    const int wg = xcd * q + min(xcd, rem) + k;
    const int wg_per_chunk = (n_runs + blockDim.x - 1) / blockDim.x;
    const int chunk = wg / wg_per_chunk;
    const int run = (wg - chunk * wg_per_chunk) * blockDim.x + threadIdx.x;
    if (run >= n_runs) return;
    const int i = run / runs_per_row;
    const int j0 = (run - i * runs_per_row) * 4;
    const int c0 = chunk * cpt;
    const int c1 = min(C, c0 + cpt);

    const int b = (i / cells) * bw + (j0 / cells);
    const int32_t vec = reinterpret_cast<const int32_t*>(mv)[b];
    const int dx = (int16_t)(vec & 0xffff), dy = (int16_t)((uint32_t)vec >> 16);
    const int ny = i * s + dy, nx = j0 * s + dx;
    const int y0 = floor_div(ny, s), x0 = floor_div(nx, s);
    const float wy = (float)(ny - y0 * s) * inv_s;
    const float wx = (float)(nx - x0 * s) * inv_s;
    const int ya = min(max(y0, 0), Hf - 1), yb = min(max(y0 + 1, 0), Hf - 1);
    int xo[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) xo[t] = min(max(x0 + t, 0), Wf - 1);
    const float w00 = (1.f - wy) * (1.f - wx), w01 = (1.f - wy) * wx;
    const float w10 = wy * (1.f - wx), w11 = wy * wx;
    const int nout = min(4, Wf - j0);
    const size_t plane = (size_t)Hf * Wf;
    const size_t ra = (size_t)ya * Wf, rb = (size_t)yb * Wf;
    const size_t obase = (size_t)i * Wf + j0;

    for (int cb = c0; cb < c1; cb += 4) {
        float va[4][5], vb[4][5];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = cb + u < c1 ? cb + u : c1 - 1;
            const size_t base = (size_t)c * plane;
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                if (BF16) {
                    const uint16_t* p = reinterpret_cast<const uint16_t*>(zin) + base;
                    va[u][t] = bf16_to_f32(p[ra + xo[t]]);
                    vb[u][t] = bf16_to_f32(p[rb + xo[t]]);
                } else {
                    const float* p = reinterpret_cast<const float*>(zin) + base;
                    va[u][t] = p[ra + xo[t]];
                    vb[u][t] = p[rb + xo[t]];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (cb + u >= c1) break;
            float o[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                float acc = w00 * va[u][t];
                acc = fmaf(w01, va[u][t + 1], acc);
                acc = fmaf(w10, vb[u][t], acc);
                acc = fmaf(w11, vb[u][t + 1], acc);
                o[t] = acc;
            }
            const size_t ob = (size_t)(cb + u) * plane + obase;
            if (BF16) {
                uint16_t* p = reinterpret_cast<uint16_t*>(zout) + ob;
                if (nout == 4 && (reinterpret_cast<uintptr_t>(p) & 7u) == 0) {
                    uint2 w;
                    w.x = (uint32_t)f32_to_bf16(o[0]) | (uint32_t)f32_to_bf16(o[1]) << 16;
                    w.y = (uint32_t)f32_to_bf16(o[2]) | (uint32_t)f32_to_bf16(o[3]) << 16;
                    *reinterpret_cast<uint2*>(p) = w;
                } else {
                    for (int t = 0; t < nout; ++t) p[t] = f32_to_bf16(o[t]);
                }
            } else {
                float* p = reinterpret_cast<float*>(zout) + ob;
                if (nout == 4 && (reinterpret_cast<uintptr_t>(p) & 15u) == 0) {
                    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
                } else {
                    for (int t = 0; t < nout; ++t) p[t] = o[t];
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_warp(const void* z, void* out, int bf16, int C, int Hf, int Wf, const int16_t* mv, int bw,
                       int cells, int s, hipStream_t stream)
{
    const float inv_s = 1.0f / (float)s;
    const int threads = 256;
    if (cells % 4 == 0) {
        // the output pointer and plane size decide whether runs can be stored
        // as one vector; the kernel checks each run's alignment itself
        const int runs_per_row = (Wf + 3) / 4;
        const int n_runs = Hf * runs_per_row;
        const int cpt = C < 8 ? C : 8;
        const int chunks = (C + cpt - 1) / cpt;
        const int wg_per_chunk = (n_runs + threads - 1) / threads;
        const long long nwg = (long long)chunks * wg_per_chunk;
        if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
        if (bf16)
            hipLaunchKernelGGL(warp_run_kernel<true>, dim3((unsigned)nwg), dim3(threads), 0, stream, z, out, C, Hf, Wf,
                               mv, bw, cells, s, inv_s, cpt, runs_per_row, n_runs);
        else
            hipLaunchKernelGGL(warp_run_kernel<false>, dim3((unsigned)nwg), dim3(threads), 0, stream, z, out, C, Hf,
                               Wf, mv, bw, cells, s, inv_s, cpt, runs_per_row, n_runs);
        return hipGetLastError();
    }
    const int ncell = Hf * Wf;
    const int cpt = C < 16 ? C : 16;
    dim3 grid((ncell + threads - 1) / threads, (C + cpt - 1) / cpt);
    if (bf16)
        hipLaunchKernelGGL(warp_kernel<true>, grid, dim3(threads), 0, stream, z, out, C, Hf, Wf, mv, bw, cells, s,
                           inv_s, cpt);
    else
        hipLaunchKernelGGL(warp_kernel<false>, grid, dim3(threads), 0, stream, z, out, C, Hf, Wf, mv, bw, cells, s,
                           inv_s, cpt);
    return hipGetLastError();
}

}  // namespace me
