// Bilinear propagation of one feature cell by its block's vector (paper
// Sec. 3.3, z_pred = Warp(z_R, MV)): the taps and weights of cell (i, j),
// shared by the warp kernel and the search kernels' fused warp epilogue so
// that both produce the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

struct WarpTaps {
    int o00, o01, o10, o11;         // plane offsets of the four neighbours
    float w00, w01, w10, w11;       // bilinear weights
};

__device__ __forceinline__ int warp_floor_div(int a, int b)
{
    const int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Cell (i, j) samples the map at (i + dy / s, j + dx / s) cells, neighbour
// indices clamped to the map.
__device__ __forceinline__ WarpTaps warp_taps(int i, int j, int dx, int dy, int s, float inv_s, int Hf, int Wf)
{
    const int ny = i * s + dy, nx = j * s + dx;
    const int y0 = warp_floor_div(ny, s), x0 = warp_floor_div(nx, s);
    const float wy = (float)(ny - y0 * s) * inv_s;
    const float wx = (float)(nx - x0 * s) * inv_s;
    const int ya = min(max(y0, 0), Hf - 1), yb = min(max(y0 + 1, 0), Hf - 1);
    const int xa = min(max(x0, 0), Wf - 1), xb = min(max(x0 + 1, 0), Wf - 1);
    WarpTaps t;
    t.w00 = (1.f - wy) * (1.f - wx);
    t.w01 = (1.f - wy) * wx;
    t.w10 = wy * (1.f - wx);
    t.w11 = wy * wx;
    t.o00 = ya * Wf + xa;
    t.o01 = ya * Wf + xb;
    t.o10 = yb * Wf + xa;
    t.o11 = yb * Wf + xb;
    return t;
}

__device__ __forceinline__ float warp_mix(const WarpTaps& t, float v00, float v01, float v10, float v11)
{
    float acc = t.w00 * v00;
    acc = fmaf(t.w01, v01, acc);
    acc = fmaf(t.w10, v10, acc);
    acc = fmaf(t.w11, v11, acc);
    return acc;
}

}  // namespace me
