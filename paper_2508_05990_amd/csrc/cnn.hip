// Proposal network of the learned-proposal mode on gfx950: forward, loss,
// backward and AdamW, all as HIP kernels (bfloat16 MFMA, float32 accumulate).
//
// Network: input = 4x4 mean of each of the four packed planes of reference
// and current frame (8 channels: the packed pair at a quarter of its
// resolution per axis), normalised to (v - 2048) / 1024; four 3x3
// convolutions, zero padding 1, strides 2, 2, 1, 1, channels
// 8 -> 32 -> 32 -> 32 -> 3, ReLU after the first three; output per 16x16
// block: (mvx, mvy) in units of 8 packed pixels and a confidence logit.
// Loss: reverse Huber (BerHu, paper Sec. 3.3; threshold one output unit,
// 8 packed pixels) on the vector, binary
// cross-entropy of the logit against "the full-search vector lies in the
// refine window of the decoded proposal"; optimiser AdamW with a cosine
// schedule (paper Sec. 4.1, training details).
//
// Layouts.  Activations are bfloat16, channels last: [n][H][W][C].  A
// convolution is an implicit GEMM with K ordered k = (ky*3 + kx) * Cin + c.
// MFMA v_mfma_f32_16x16x16_bf16 takes, per lane L (g = L / 16): A[m = L%16]
// [k = 4g..4g+3], B[k = 4g..4g+3][n = L%16], and returns D[m = 4g+i][n = L%16].
// A wave computes 16 output pixels (the n index) for every output channel (m).
// Weights are repacked after each update into the A-operand order, once for
// the forward GEMM (m = out channel) and once for the input-gradient GEMM
// (m = in channel, k = tap * Coutp + out channel).  Weight gradients reduce
// over pixels in LDS-staged chunks into per-workgroup partials that a second
// kernel sums in a fixed order: no float atomics, so training is
// bit-reproducible.
#include "bf16.h"
#include "internal.h"

namespace me {
namespace {

// ---------------------------------------------------------------- pooling --

// out[y][x][c]: c < 4 from ref, c >= 4 from cur; plane c of a mosaic is
// sample (2py + (c>>1), 2px + (c&1)), and output pixel (y, x) averages packed
// pixels (4y..4y+3, 4x..4x+3), i.e. the 16 samples of colour c in the 8 x 8
// mosaic cell at rows 8y.., columns 8x..: rows 8y + (c>>1) + {0,2,4,6},
// columns 8x + (c&1) + {0,2,4,6}.  Sums are exact integers; the mean is
// scaled by a power of two, so the only rounding is the final bfloat16 one.
__global__ void pool_kernel(const uint16_t* __restrict__ ref, int64_t ref_pitch, const uint16_t* __restrict__ cur,
                            int64_t cur_pitch, int Hq, int Wq, uint16_t* __restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Hq * Wq) return;
    const int y = p / Wq, x = p - y * Wq;
    float v[8];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const uint16_t* m = f ? cur : ref;
        const int64_t pitch = f ? cur_pitch : ref_pitch;
        // per mosaic row of the cell, the sums of its even and odd columns
        uint32_t se[8], so[8];
        if ((pitch & 7) == 0 && (reinterpret_cast<uintptr_t>(m) & 15) == 0) {
            uint4 u[8];                                   // one 16-byte load per row, all issued first
#pragma unroll
            for (int r = 0; r < 8; ++r) u[r] = *reinterpret_cast<const uint4*>(m + (8LL * y + r) * pitch + 8LL * x);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                se[r] = (u[r].x & 0xffffu) + (u[r].y & 0xffffu) + (u[r].z & 0xffffu) + (u[r].w & 0xffffu);
                so[r] = (u[r].x >> 16) + (u[r].y >> 16) + (u[r].z >> 16) + (u[r].w >> 16);
            }
        } else {
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const uint16_t* row = m + (8LL * y + r) * pitch + 8LL * x;
                se[r] = (uint32_t)row[0] + row[2] + row[4] + row[6];
                so[r] = (uint32_t)row[1] + row[3] + row[5] + row[7];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int r0 = c >> 1;
            const uint32_t* cs = (c & 1) ? so : se;
            const uint32_t s = cs[r0] + cs[r0 + 2] + cs[r0 + 4] + cs[r0 + 6];
            v[4 * f + c] = ((float)s * 0.0625f - 2048.0f) * (1.0f / 1024.0f);
        }
    }
    uint4 w;
    w.x = (uint32_t)f2bf(v[0]) | (uint32_t)f2bf(v[1]) << 16;
    w.y = (uint32_t)f2bf(v[2]) | (uint32_t)f2bf(v[3]) << 16;
    w.z = (uint32_t)f2bf(v[4]) | (uint32_t)f2bf(v[5]) << 16;
    w.w = (uint32_t)f2bf(v[6]) | (uint32_t)f2bf(v[7]) << 16;
    reinterpret_cast<uint4*>(out)[p] = w;
}

// ------------------------------------------------------------ parameters --

struct LayerDesc {
    int cin, cout, stride, off_w, off_b;
};

__constant__ LayerDesc kLayers[4] = {
    {8, 32, 2, 0, 2304}, {32, 32, 2, 2336, 11552}, {32, 32, 1, 11584, 20800}, {32, 3, 1, 20832, 21696}};

// Forward A operand of layer l: [mt][ks][lane][4], m = out channel, k = tap*cin + c.
// Input-gradient A operand: [ct][ks][lane][4], m = in channel, k = tap*coutp + o.
__device__ __host__ inline int packed_fwd(int cin, int cout) { return ((cout + 15) / 16) * ((9 * cin + 15) / 16) * 256; }
__device__ __host__ inline int packed_bwd(int cin, int cout)
{
    return ((cin + 15) / 16) * ((9 * ((cout + 3) & ~3) + 15) / 16) * 256;
}

__global__ void pack_kernel(const float* __restrict__ w, uint16_t* __restrict__ fwd, uint16_t* __restrict__ bwd)
{
    const int l = blockIdx.y;
    const LayerDesc L = kLayers[l];
    int fo = 0, bo = 0;
    for (int j = 0; j < l; ++j) {
        fo += packed_fwd(kLayers[j].cin, kLayers[j].cout);
        bo += packed_bwd(kLayers[j].cin, kLayers[j].cout);
    }
    const int K = 9 * L.cin, ksteps = (K + 15) / 16, mt = (L.cout + 15) / 16;
    const int coutp = (L.cout + 3) & ~3;
    const int Kb = 9 * coutp, kbsteps = (Kb + 15) / 16, ct = (L.cin + 15) / 16;
    const int nf = mt * ksteps * 256, nb = ct * kbsteps * 256;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nf + nb; e += gridDim.x * blockDim.x) {
        if (e < nf) {
            const int j = e & 3, lane = (e >> 2) & 63, ks = (e >> 8) % ksteps, t = (e >> 8) / ksteps;
            const int o = t * 16 + (lane & 15), k = ks * 16 + 4 * (lane >> 4) + j;
            float v = 0.f;
            if (o < L.cout && k < K) {
                const int tap = k / L.cin, c = k - tap * L.cin;
                v = w[L.off_w + (o * L.cin + c) * 9 + tap];
            }
            fwd[fo + e] = f2bf(v);
        } else {
            const int e2 = e - nf;
            const int j = e2 & 3, lane = (e2 >> 2) & 63, ks = (e2 >> 8) % kbsteps, t = (e2 >> 8) / kbsteps;
            const int c = t * 16 + (lane & 15), k = ks * 16 + 4 * (lane >> 4) + j;
            float v = 0.f;
            if (c < L.cin && k < Kb) {
                const int tap = k / coutp, o = k - tap * coutp;
                if (o < L.cout) v = w[L.off_w + (o * L.cin + c) * 9 + tap];
            }
            bwd[bo + e2] = f2bf(v);
        }
    }
}

// --------------------------------------------------------------- forward --

// One wave = 16 output pixels of the flattened [n][Ho][Wo]; 4 waves per
// workgroup.  LAST: float32 output [n][COUT][Ho][Wo] without ReLU; otherwise
// bfloat16 [n][Ho][Wo][COUT] after ReLU.
template <int CIN, int COUT, int S, bool LAST>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wp,
                                                       const float* __restrict__ bias, void* __restrict__ out, int n,
                                                       int H, int W, int Ho, int Wo)
{
    constexpr int K = 9 * CIN, KS = (K + 15) / 16, MT = (COUT + 15) / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4;
    const int P = n * Ho * Wo;
    const int p = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + (lane & 15);
    const bool valid = p < P;
    const int pp = valid ? p : 0;
    const int img = pp / (Ho * Wo), rem = pp - img * Ho * Wo;
    const int oy = rem / Wo, ox = rem - oy * Wo;
    const uint16_t* src = in + (size_t)img * H * W * CIN;

    v4f32 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k0 = ks * 16 + 4 * g;
        uint2 bv = make_uint2(0u, 0u);
        if (k0 < K) {
            const int tap = k0 / CIN, c = k0 - tap * CIN;
            const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
            if (iy >= 0 && iy < H && ix >= 0 && ix < W)
                bv = *reinterpret_cast<const uint2*>(src + ((size_t)iy * W + ix) * CIN + c);
        }
        const v4i16 b = as_v4(bv);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const uint2 av = reinterpret_cast<const uint2*>(wp)[(t * KS + ks) * 64 + lane];
            acc[t] = mfma(as_v4(av), b, acc[t]);
        }
    }
    if (!valid) return;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int o0 = t * 16 + 4 * g;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = acc[t][i] + (o0 + i < COUT ? bias[o0 + i] : 0.f);
        if (LAST) {
            float* o = reinterpret_cast<float*>(out) + (size_t)img * COUT * Ho * Wo + rem;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (o0 + i < COUT) o[(size_t)(o0 + i) * Ho * Wo] = v[i];
        } else {
            uint16_t* o = reinterpret_cast<uint16_t*>(out) + (size_t)pp * COUT + o0;
            *reinterpret_cast<uint2*>(o) = pack4(fmaxf(v[0], 0.f), fmaxf(v[1], 0.f), fmaxf(v[2], 0.f), fmaxf(v[3], 0.f));
        }
    }
}

// Split-k variant for small grids: a workgroup's four waves take the same 16
// output pixels and the k-steps w, w + 4, ... each; the partial sums meet in
// LDS and wave 0 adds them in wave order (a fixed order: results stay
// reproducible), then stores as conv_fwd_kernel does.  Four times the waves and
// a quarter of each wave's chain of dependent products.
template <int CIN, int COUT, int S, bool LAST>
__global__ __launch_bounds__(256) void conv_fwd_split_kernel(const uint16_t* __restrict__ in,
                                                             const uint16_t* __restrict__ wp,
                                                             const float* __restrict__ bias, void* __restrict__ out,
                                                             int n, int H, int W, int Ho, int Wo)
{
    constexpr int K = 9 * CIN, KS = (K + 15) / 16, MT = (COUT + 15) / 16;
    __shared__ v4f32 part[3][MT][64];
    const int lane = threadIdx.x & 63, g = lane >> 4, w = threadIdx.x >> 6;
    const int P = n * Ho * Wo;
    const int p = blockIdx.x * 16 + (lane & 15);
    const bool valid = p < P;
    const int pp = valid ? p : 0;
    const int img = pp / (Ho * Wo), rem = pp - img * Ho * Wo;
    const int oy = rem / Wo, ox = rem - oy * Wo;
    const uint16_t* src = in + (size_t)img * H * W * CIN;

    v4f32 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < (KS + 3) / 4; ++j) {
        const int ks = 4 * j + w;
        if (ks >= KS) break;
        const int k0 = ks * 16 + 4 * g;
        uint2 bv = make_uint2(0u, 0u);
        if (k0 < K) {
            const int tap = k0 / CIN, c = k0 - tap * CIN;
            const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
            if (iy >= 0 && iy < H && ix >= 0 && ix < W)
                bv = *reinterpret_cast<const uint2*>(src + ((size_t)iy * W + ix) * CIN + c);
        }
        const v4i16 b = as_v4(bv);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const uint2 av = reinterpret_cast<const uint2*>(wp)[(t * KS + ks) * 64 + lane];
            acc[t] = mfma(as_v4(av), b, acc[t]);
        }
    }
    if (w > 0) {
#pragma unroll
        for (int t = 0; t < MT; ++t) part[w - 1][t][lane] = acc[t];
    }
    __syncthreads();
    if (w != 0 || !valid) return;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        acc[t] = acc[t] + part[0][t][lane];
        acc[t] = acc[t] + part[1][t][lane];
        acc[t] = acc[t] + part[2][t][lane];
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int o0 = t * 16 + 4 * g;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = acc[t][i] + (o0 + i < COUT ? bias[o0 + i] : 0.f);
        if (LAST) {
            float* o = reinterpret_cast<float*>(out) + (size_t)img * COUT * Ho * Wo + rem;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (o0 + i < COUT) o[(size_t)(o0 + i) * Ho * Wo] = v[i];
        } else {
            uint16_t* o = reinterpret_cast<uint16_t*>(out) + (size_t)pp * COUT + o0;
            *reinterpret_cast<uint2*>(o) = pack4(fmaxf(v[0], 0.f), fmaxf(v[1], 0.f), fmaxf(v[2], 0.f), fmaxf(v[3], 0.f));
        }
    }
}

// ------------------------------------------------------------------ loss --

__device__ __forceinline__ float berhu(float x, float c) { const float a = fabsf(x); return a <= c ? a : (x * x + c * c) / (2.f * c); }
__device__ __forceinline__ float berhu_grad(float x, float c) { return fabsf(x) <= c ? (x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f)) : x / c; }

// Per block: loss value and the gradient of the batch mean, as bfloat16
// [n][nblk][4] (channel 3 = 0) for the last layer's backward.
__global__ void loss_kernel(const float* __restrict__ out, const int16_t* __restrict__ mv,
                            const float* __restrict__ wt, int n, int nblk, int R, int rr, float scale,
                            uint16_t* __restrict__ dz, float* __restrict__ bl)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nblk) return;
    const int img = e / nblk, b = e - img * nblk;
    const float* o = out + (size_t)img * 3 * nblk;
    const float ox = o[b], oy = o[nblk + b], lg = o[2 * nblk + b];
    const int mx = mv[2 * e], my = mv[2 * e + 1];
    const float r = (float)R;
    const float px = fminf(fmaxf(rintf(8.f * ox), -r), r), py = fminf(fmaxf(rintf(8.f * oy), -r), r);
    const float dmax = fmaxf(fabsf(px - (float)mx), fabsf(py - (float)my));
    const float y = dmax <= (float)rr ? 1.f : 0.f;
    const float c = 1.0f;                          // one output unit = 8 packed pixels
    const float ex = ox - (float)mx * 0.125f, ey = oy - (float)my * 0.125f;
    const float bce = fmaxf(lg, 0.f) - lg * y + log1pf(expf(-fabsf(lg)));
    const float w = wt ? wt[e] : 1.f;              // weight of the vector term
    bl[e] = w * (berhu(ex, c) + berhu(ey, c)) + bce;
    const float sg = lg >= 0.f ? 1.f / (1.f + expf(-lg)) : expf(lg) / (1.f + expf(lg));
    *reinterpret_cast<uint2*>(dz + 4 * (size_t)e) =
        pack4(w * berhu_grad(ex, c) * scale, w * berhu_grad(ey, c) * scale, (sg - y) * scale, 0.f);
}

// Fixed-order sum of the block losses, times scale (one workgroup).
__global__ void loss_sum_kernel(const float* __restrict__ bl, int m, float scale, float* __restrict__ loss)
{
    __shared__ double part[256];
    double s = 0.0;
    for (int e = threadIdx.x; e < m; e += blockDim.x) s += (double)bl[e];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)blockDim.x; ++k) t += part[k];
        *loss = (float)(t * (double)scale);
    }
}

// -------------------------------------------------------- input gradient --

// dX for layer with (CIN, COUTP, S): one wave = 16 input pixels of the
// flattened [n][H][W]; k = tap * COUTP + o gathers dZ at the output pixel
// that tap (ky, kx) of the input pixel contributes to.  The result is masked
// by the ReLU of the previous layer (its stored output > 0) and stored as
// that layer's output gradient, bfloat16 [n][H][W][CIN].
template <int CIN, int COUTP, int S>
__global__ __launch_bounds__(256) void conv_dgrad_kernel(const uint16_t* __restrict__ dz,
                                                         const uint16_t* __restrict__ wb,
                                                         const uint16_t* __restrict__ aprev,
                                                         uint16_t* __restrict__ dprev, int n, int H, int W, int Ho,
                                                         int Wo)
{
    constexpr int K = 9 * COUTP, KS = (K + 15) / 16, CT = (CIN + 15) / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4;
    const int P = n * H * W;
    const int p = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + (lane & 15);
    const bool valid = p < P;
    const int pp = valid ? p : 0;
    const int img = pp / (H * W), rem = pp - img * H * W;
    const int iy = rem / W, ix = rem - iy * W;
    const uint16_t* src = dz + (size_t)img * Ho * Wo * COUTP;

    v4f32 acc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[t] = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k0 = ks * 16 + 4 * g;
        uint2 bv = make_uint2(0u, 0u);
        if (k0 < K) {
            const int tap = k0 / COUTP, o = k0 - tap * COUTP;
            const int ny = iy + 1 - tap / 3, nx = ix + 1 - tap % 3;
            if (ny >= 0 && nx >= 0 && ny % S == 0 && nx % S == 0) {
                const int oy = ny / S, ox = nx / S;
                if (oy < Ho && ox < Wo) bv = *reinterpret_cast<const uint2*>(src + ((size_t)oy * Wo + ox) * COUTP + o);
            }
        }
        const v4i16 b = as_v4(bv);
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const uint2 av = reinterpret_cast<const uint2*>(wb)[(t * KS + ks) * 64 + lane];
            acc[t] = mfma(as_v4(av), b, acc[t]);
        }
    }
    if (!valid) return;
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int c0 = t * 16 + 4 * g;
        if (c0 >= CIN) continue;
        const uint2 av = *reinterpret_cast<const uint2*>(aprev + (size_t)pp * CIN + c0);
        const float m0 = bf2f(av.x & 0xffffu), m1 = bf2f(av.x >> 16);
        const float m2 = bf2f(av.y & 0xffffu), m3 = bf2f(av.y >> 16);
        *reinterpret_cast<uint2*>(dprev + (size_t)pp * CIN + c0) =
            pack4(m0 > 0.f ? acc[t][0] : 0.f, m1 > 0.f ? acc[t][1] : 0.f, m2 > 0.f ? acc[t][2] : 0.f,
                  m3 > 0.f ? acc[t][3] : 0.f);
    }
}

// ------------------------------------------------------- weight gradient --

// Partial dW[o][k] and db[o] of one workgroup over `chunks` chunks of 64
// output pixels (flattened [n][Ho][Wo]), chunk c handled by workgroup
// c % gridDim.x.  The chunk's im2col of the layer input (k-major) and its dZ
// (channel-major) are staged in LDS; D[o][k] += dZ[o][p] X[k][p] on MFMA with
// the 64 pixels as the reduction dimension.
template <int CIN, int COUT, int COUTP, int S>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dz,
                                                         float* __restrict__ partial, int n, int H, int W, int Ho,
                                                         int Wo)
{
    constexpr int K = 9 * CIN, KT = (K + 15) / 16, MT = (COUT + 15) / 16;
    constexpr int PITCH = 64 + 4;                 // bf16 per LDS row (pixels)
    constexpr int TILES = MT * KT, TPW = (TILES + 3) / 4;
    __shared__ uint16_t xs[KT * 16][PITCH];
    __shared__ uint16_t ds[MT * 16][PITCH];
    __shared__ float bsum[MT * 16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4;
    const int P = n * Ho * Wo;
    const int nchunks = (P + 63) / 64;

    v4f32 acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = (v4f32){0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;                             // thread o < COUT: bias partial

    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        __syncthreads();
        // stage: xs[k][q] for k in [0, KT*16), q in [0, 64); 4 channels per item
        for (int e = tid; e < (KT * 16 / 4) * 64; e += 256) {
            const int q = e & 63, kq = e >> 6;
            const int k0 = kq * 4;
            const int p = ch * 64 + q;
            uint2 v = make_uint2(0u, 0u);
            if (p < P && k0 < K) {
                const int img = p / (Ho * Wo), rem = p - img * Ho * Wo;
                const int oy = rem / Wo, ox = rem - oy * Wo;
                const int tap = k0 / CIN, c = k0 - tap * CIN;
                const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
                if (iy >= 0 && iy < H && ix >= 0 && ix < W)
                    v = *reinterpret_cast<const uint2*>(x + (((size_t)img * H + iy) * W + ix) * CIN + c);
            }
            xs[k0 + 0][q] = (uint16_t)(v.x & 0xffff);
            xs[k0 + 1][q] = (uint16_t)(v.x >> 16);
            xs[k0 + 2][q] = (uint16_t)(v.y & 0xffff);
            xs[k0 + 3][q] = (uint16_t)(v.y >> 16);
        }
        for (int e = tid; e < (MT * 16 / 4) * 64; e += 256) {
            const int q = e & 63, oq = e >> 6;
            const int o0 = oq * 4;
            const int p = ch * 64 + q;
            uint2 v = make_uint2(0u, 0u);
            if (p < P && o0 < COUTP) v = *reinterpret_cast<const uint2*>(dz + (size_t)p * COUTP + o0);
            ds[o0 + 0][q] = (uint16_t)(v.x & 0xffff);
            ds[o0 + 1][q] = (uint16_t)(v.x >> 16);
            ds[o0 + 2][q] = (uint16_t)(v.y & 0xffff);
            ds[o0 + 3][q] = (uint16_t)(v.y >> 16);
        }
        __syncthreads();
        if (tid < COUT) {
            for (int q = 0; q < 64; ++q) bacc += bf2f(ds[tid][q]);
        }
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int tile = wave + 4 * t;
            if (tile < TILES) {
                const int mt = tile / KT, kt = tile - mt * KT;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const uint2 av = *reinterpret_cast<const uint2*>(&ds[mt * 16 + (lane & 15)][kk * 16 + 4 * g]);
                    const uint2 bv = *reinterpret_cast<const uint2*>(&xs[kt * 16 + (lane & 15)][kk * 16 + 4 * g]);
                    acc[t] = mfma(as_v4(av), as_v4(bv), acc[t]);
                }
            }
        }
    }
    // partial layout: [wg][COUT][K] then [wg] bias block [COUT] after all weight partials
    float* pw = partial + (size_t)blockIdx.x * COUT * K;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int tile = wave + 4 * t;
        if (tile < TILES) {
            const int mt = tile / KT, kt = tile - mt * KT;
            const int k = kt * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = mt * 16 + 4 * g + i;
                if (o < COUT && k < K) pw[o * K + k] = acc[t][i];
            }
        }
    }
    if (tid < COUT) partial[(size_t)gridDim.x * COUT * K + (size_t)blockIdx.x * COUT + tid] = bacc;
}

// grads (flat layout: W[o][c][ky][kx] then b[o]) = sum over workgroups of the
// partials, in workgroup order.
__global__ void wgrad_reduce_kernel(const float* __restrict__ partial, int nwg, int cin, int cout, int off_w,
                                    int off_b, float* __restrict__ grads)
{
    const int K = 9 * cin;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < cout * K) {
        const int o = e / K, k = e - o * K;
        float s = 0.f;
        for (int w = 0; w < nwg; ++w) s += partial[(size_t)w * cout * K + e];
        const int tap = k / cin, c = k - tap * cin;
        grads[off_w + (o * cin + c) * 9 + tap] = s;
    } else if (e < cout * K + cout) {
        const int o = e - cout * K;
        float s = 0.f;
        for (int w = 0; w < nwg; ++w) s += partial[(size_t)nwg * cout * K + (size_t)w * cout + o];
        grads[off_b + o] = s;
    }
}

// ----------------------------------------------------------------- AdamW --

__global__ void adamw_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, int np, float lr, float b1, float b2, float eps, float wd, float c1,
                             float c2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= np) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float mh = mi * c1, vh = vi * c2;
    const float wi = w[e];
    w[e] = wi - lr * (mh / (sqrtf(vh) + eps) + wd * wi);
}

int div_up(int a, int b) { return (a + b - 1) / b; }

}  // namespace

// ------------------------------------------------------------ host side --

static const int kCin[4] = {8, 32, 32, 32}, kCout[4] = {32, 32, 32, 3};

int cnn_fwd_packed_size(int l) { return packed_fwd(kCin[l], kCout[l]); }
int cnn_bwd_packed_size(int l) { return packed_bwd(kCin[l], kCout[l]); }

hipError_t launch_pool(const uint16_t* ref, int64_t ref_pitch, const uint16_t* cur, int64_t cur_pitch, int Hq, int Wq,
                       uint16_t* out, hipStream_t st)
{
    const int np = Hq * Wq;
    hipLaunchKernelGGL(pool_kernel, dim3(div_up(np, 256)), dim3(256), 0, st, ref, ref_pitch, cur, cur_pitch, Hq, Wq,
                       out);
    return hipGetLastError();
}

hipError_t launch_pack(const float* w, uint16_t* fwd, uint16_t* bwd, hipStream_t st)
{
    hipLaunchKernelGGL(pack_kernel, dim3(64, 4), dim3(256), 0, st, w, fwd, bwd);
    return hipGetLastError();
}

hipError_t launch_conv_fwd(int l, const uint16_t* in, const uint16_t* wp, const float* bias, void* out, int n, int H,
                           int W, int Ho, int Wo, hipStream_t st)
{
    const int P = n * Ho * Wo;
    dim3 grid(div_up(P, 64)), blk(256);
    if (div_up(P, 64) < 1024) {   // small grid: split the k-steps over the workgroup's waves
        const dim3 sg(div_up(P, 16));
        switch (l) {
        case 0: hipLaunchKernelGGL((conv_fwd_split_kernel<8, 32, 2, false>), sg, blk, 0, st, in, wp, bias, out, n, H, W, Ho, Wo); break;
        case 1: hipLaunchKernelGGL((conv_fwd_split_kernel<32, 32, 2, false>), sg, blk, 0, st, in, wp, bias, out, n, H, W, Ho, Wo); break;
        case 2: hipLaunchKernelGGL((conv_fwd_split_kernel<32, 32, 1, false>), sg, blk, 0, st, in, wp, bias, out, n, H, W, Ho, Wo); break;
        case 3: hipLaunchKernelGGL((conv_fwd_split_kernel<32, 3, 1, true>), sg, blk, 0, st, in, wp, bias, out, n, H, W, Ho, Wo); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (l) {
    case 0: hipLaunchKernelGGL((conv_fwd_kernel<8, 32, 2, false>), grid, blk, 0, st, in, wp, bias, out, n, H, W, Ho, Wo); break;
    case 1: hipLaunchKernelGGL((conv_fwd_kernel<32, 32, 2, false>), grid, blk, 0, st, in, wp, bias, out, n, H, W, Ho, Wo); break;
    case 2: hipLaunchKernelGGL((conv_fwd_kernel<32, 32, 1, false>), grid, blk, 0, st, in, wp, bias, out, n, H, W, Ho, Wo); break;
    case 3: hipLaunchKernelGGL((conv_fwd_kernel<32, 3, 1, true>), grid, blk, 0, st, in, wp, bias, out, n, H, W, Ho, Wo); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_loss(const float* out, const int16_t* mv, const float* wt, int n, int nblk, int R, int rr,
                       uint16_t* dz, float* bl, float* loss, hipStream_t st)
{
    const int m = n * nblk;
    const float scale = 1.0f / (float)m;
    hipLaunchKernelGGL(loss_kernel, dim3(div_up(m, 256)), dim3(256), 0, st, out, mv, wt, n, nblk, R, rr, scale, dz,
                       bl);
    if (loss) hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, st, bl, m, scale, loss);
    return hipGetLastError();
}

// Input gradient of layer l (l = 1, 2, 3) masked by layer l-1's ReLU.
hipError_t launch_conv_dgrad(int l, const uint16_t* dz, const uint16_t* wb, const uint16_t* aprev, uint16_t* dprev,
                             int n, int H, int W, int Ho, int Wo, hipStream_t st)
{
    const int P = n * H * W;
    dim3 grid(div_up(P, 64)), blk(256);
    switch (l) {
    case 1: hipLaunchKernelGGL((conv_dgrad_kernel<32, 32, 2>), grid, blk, 0, st, dz, wb, aprev, dprev, n, H, W, Ho, Wo); break;
    case 2: hipLaunchKernelGGL((conv_dgrad_kernel<32, 32, 1>), grid, blk, 0, st, dz, wb, aprev, dprev, n, H, W, Ho, Wo); break;
    case 3: hipLaunchKernelGGL((conv_dgrad_kernel<32, 4, 1>), grid, blk, 0, st, dz, wb, aprev, dprev, n, H, W, Ho, Wo); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int cnn_wgrad_groups(int n, int Ho, int Wo)
{
    const int chunks = div_up(n * Ho * Wo, 64);
    return chunks < 256 ? chunks : 256;
}

size_t cnn_wgrad_partial_floats(int l, int nwg) { return (size_t)nwg * kCout[l] * (9 * kCin[l] + 1); }

// Weight and bias gradients of layer l into `grads` (flat layout).
hipError_t launch_conv_wgrad(int l, const uint16_t* x, const uint16_t* dz, float* partial, float* grads, int n, int H,
                             int W, int Ho, int Wo, hipStream_t st)
{
    static const int offw[4] = {0, 2336, 11584, 20832}, offb[4] = {2304, 11552, 20800, 21696};
    const int* cin = kCin;
    const int* cout = kCout;
    const int nwg = cnn_wgrad_groups(n, Ho, Wo);
    dim3 grid(nwg), blk(256);
    switch (l) {
    case 0: hipLaunchKernelGGL((conv_wgrad_kernel<8, 32, 32, 2>), grid, blk, 0, st, x, dz, partial, n, H, W, Ho, Wo); break;
    case 1: hipLaunchKernelGGL((conv_wgrad_kernel<32, 32, 32, 2>), grid, blk, 0, st, x, dz, partial, n, H, W, Ho, Wo); break;
    case 2: hipLaunchKernelGGL((conv_wgrad_kernel<32, 32, 32, 1>), grid, blk, 0, st, x, dz, partial, n, H, W, Ho, Wo); break;
    case 3: hipLaunchKernelGGL((conv_wgrad_kernel<32, 3, 4, 1>), grid, blk, 0, st, x, dz, partial, n, H, W, Ho, Wo); break;
    default: return hipErrorInvalidValue;
    }
    const int m = cout[l] * 9 * cin[l] + cout[l];
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(div_up(m, 256)), dim3(256), 0, st, partial, nwg, cin[l], cout[l],
                       offw[l], offb[l], grads);
    return hipGetLastError();
}

hipError_t launch_adamw(float* w, const float* g, float* m, float* v, int np, float lr, float b1, float b2, float eps,
                        float wd, float c1, float c2, hipStream_t st)
{
    hipLaunchKernelGGL(adamw_kernel, dim3(div_up(np, 256)), dim3(256), 0, st, w, g, m, v, np, lr, b1, b2, eps, wd, c1,
                       c2);
    return hipGetLastError();
}

}  // namespace me
