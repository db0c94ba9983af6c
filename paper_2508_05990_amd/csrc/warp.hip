// Propagation of a reference feature map by per-block motion vectors,
// z_pred = Warp(z_R, MV) (paper Sec. 3.3), on gfx950.
//
// HBM-bound: every output element reads four neighbouring inputs (mostly
// L2/L1 hits, since neighbouring cells of a block share one vector) and is
// written once.  The vector, the clamped row and column indices and the four
// bilinear weights are computed once per thread and reused for every channel
// of its chunk; consecutive lanes take consecutive cells of a row, so loads
// and stores of a channel plane are contiguous across the wave.
#include "bf16.h"
#include "internal.h"
#include "warp_cell.h"

namespace me {
namespace {

// One cell per lane (consecutive lanes, consecutive cells: every load and
// store instruction of a wave covers a contiguous stretch of a plane) and a
// chunk of channels per thread, four channels' loads in flight before use.
template <bool BF16>
__global__ __launch_bounds__(256) void warp_kernel(const void* __restrict__ zin, void* __restrict__ zout, int C,
                                                   int Hf, int Wf, const int16_t* __restrict__ mv, int bw, int cells,
                                                   int s, float inv_s, int cpt, int wg_per_chunk)
{
    // work item = (channel chunk, cell); XCD-contiguous ranges of items so the
    // rows a chunk shares between neighbouring workgroups stay in one L2
    const int nwg = gridDim.x;
    const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
    const int q = nwg >> 3, rem = nwg & 7;
    const int wg = xcd * q + min(xcd, rem) + k;
    const int chunk = wg / wg_per_chunk;
    const int cell = (wg - chunk * wg_per_chunk) * blockDim.x + threadIdx.x;
    const int ncell = Hf * Wf;
    if (cell >= ncell) return;
    const int i = cell / Wf, j = cell - i * Wf;
    const int c0 = chunk * cpt;
    const int c1 = min(C, c0 + cpt);

    const int b = (i / cells) * bw + (j / cells);
    const int32_t vec = reinterpret_cast<const int32_t*>(mv)[b];   // (dx, dy) as two int16
    const int dx = (int16_t)(vec & 0xffff), dy = (int16_t)((uint32_t)vec >> 16);
    const WarpTaps tp = warp_taps(i, j, dx, dy, s, inv_s, Hf, Wf);
    const int o00 = tp.o00, o01 = tp.o01, o10 = tp.o10, o11 = tp.o11;

    const size_t plane = (size_t)ncell;
    for (int cb = c0; cb < c1; cb += 4) {
        float v[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = cb + u < c1 ? cb + u : c1 - 1;
            const size_t base = (size_t)c * plane;
            if (BF16) {
                const uint16_t* p = reinterpret_cast<const uint16_t*>(zin) + base;
                v[u][0] = bf2f(p[o00]);
                v[u][1] = bf2f(p[o01]);
                v[u][2] = bf2f(p[o10]);
                v[u][3] = bf2f(p[o11]);
            } else {
                const float* p = reinterpret_cast<const float*>(zin) + base;
                v[u][0] = p[o00];
                v[u][1] = p[o01];
                v[u][2] = p[o10];
                v[u][3] = p[o11];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (cb + u >= c1) break;
            const float acc = warp_mix(tp, v[u][0], v[u][1], v[u][2], v[u][3]);
            const size_t o = (size_t)(cb + u) * plane + cell;
            // the output is written once and not read back here: non-temporal stores
            if (BF16)
                __builtin_nontemporal_store(f2bf(acc), reinterpret_cast<uint16_t*>(zout) + o);
            else
                __builtin_nontemporal_store(acc, reinterpret_cast<float*>(zout) + o);
        }
    }
}

// Chain block vectors over a group of pictures: block b's centre displaced
// by its step vector falls in block b' of the previous frame, whose vector to
// the key frame is added.  One thread per block; out may alias ms (each
// thread reads only its own step vector) but not ma.
__global__ void compose_kernel(const int16_t* __restrict__ ms, const int16_t* ma, int16_t* out, int bh, int bw,
                               int B, int Hp, int Wp)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bh * bw) return;
    const int bi = b / bw, bj = b - bi * bw;
    const int h = min(B, Hp - bi * B), w = min(B, Wp - bj * B);
    const int vx = ms[2 * b], vy = ms[2 * b + 1];
    const int px = bj * B + w / 2 + vx, py = bi * B + h / 2 + vy;
    const int fi = py >= 0 ? py / B : -((-py + B - 1) / B);
    const int fj = px >= 0 ? px / B : -((-px + B - 1) / B);
    const int pi = min(max(fi, 0), bh - 1), pj = min(max(fj, 0), bw - 1);
    const int pb = pi * bw + pj;
    out[2 * b] = (int16_t)(vx + ma[2 * pb]);
    out[2 * b + 1] = (int16_t)(vy + ma[2 * pb + 1]);
}

}  // namespace

hipError_t launch_compose(const int16_t* ms, const int16_t* ma, int16_t* out, int bh, int bw, int B, int Hp, int Wp,
                          hipStream_t stream)
{
    const int n = bh * bw;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(compose_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, ms, ma, out, bh, bw, B, Hp, Wp);
    return hipGetLastError();
}

hipError_t launch_warp(const void* z, void* out, int bf16, int C, int Hf, int Wf, const int16_t* mv, int bw,
                       int cells, int s, hipStream_t stream)
{
    const float inv_s = 1.0f / (float)s;
    const int threads = 256;
    const int ncell = Hf * Wf;
    const int cpt = C < 16 ? C : 16;
    const int chunks = (C + cpt - 1) / cpt;
    const int wg_per_chunk = (ncell + threads - 1) / threads;
    const long long nwg = (long long)chunks * wg_per_chunk;
    if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
    if (bf16)
        hipLaunchKernelGGL(warp_kernel<true>, dim3((unsigned)nwg), dim3(threads), 0, stream, z, out, C, Hf, Wf, mv, bw,
                           cells, s, inv_s, cpt, wg_per_chunk);
    else
        hipLaunchKernelGGL(warp_kernel<false>, dim3((unsigned)nwg), dim3(threads), 0, stream, z, out, C, Hf, Wf, mv,
                           bw, cells, s, inv_s, cpt, wg_per_chunk);
    return hipGetLastError();
}

}  // namespace me
