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

// ------------------------------------------------- whole-network forward --

// Inference forward of all four layers in one launch.  A workgroup owns a
// tile of FTY x FTX output blocks of one image and works backwards to the
// regions each layer needs (zero padding 1 at every layer): layer 2 outputs
// (FTY + 2) x (FTX + 2), layer 1 (FTY + 4) x (FTX + 4), layer 0 twice that plus
// one, the pooled input twice that plus one; all of them live in LDS,
// channels last (pixel strides padded against bank conflicts), with positions
// outside a layer's grid stored as zero (the next layer's padding).  Each layer is an implicit GEMM on MFMA whose work
// items are (16-pixel tile, 16-channel group) pairs dealt to the eight waves;
// every output takes the k-steps in order and the bias, ReLU and bfloat16
// rounding of conv_fwd_kernel, so the result equals the layer-by-layer
// chain of that kernel bit for bit.  ACTS: also store each layer's
// activations over the tile's own region (every position is owned by one
// tile), in the layer kernels' layouts.
constexpr int FTY = 2, FTX = 4;                              // output blocks per workgroup
constexpr int FNW = 8;                                       // waves per workgroup
// LDS pixel strides (bfloat16 elements, multiples of 4 for 8-byte reads),
// padded so that a wave's 16 pixels of one B-operand read fall on distinct
// banks: the reader of s_in and s_0 steps two pixels per lane (stride 2),
// the readers of s_1 and s_2 one pixel.
constexpr int PIN = 12, P0 = 36, P1 = 40, P2 = 40;
constexpr int F2Y = FTY + 2, F2X = FTX + 2;                  // layer 2 outputs needed
constexpr int F1Y = FTY + 4, F1X = FTX + 4;                  // layer 1 outputs
constexpr int F0Y = 2 * F1Y + 1, F0X = 2 * F1X + 1;          // layer 0 outputs
constexpr int FIY = 2 * F0Y + 1, FIX = 2 * F0X + 1;          // pooled input

// Layer of CIN -> COUT (ReLU, bfloat16) from an LDS region [.][IX][CIN] to an
// LDS region [OY][OX][COUT]: output (ly, lx) reads input (S ly + ky, S lx + kx).
// (gy0, gx0): grid position of output (0, 0); outputs outside [0, Ho) x [0, Wo)
// are stored as zero.
// The A operands of every k-step of 16-channel group t of a layer (KS steps)
// and the lane's four output-channel biases, requested before the barrier
// that precedes the layer so that their latency overlaps the wait.
template <int KS>
__device__ __forceinline__ void fused_operands(const uint16_t* __restrict__ wp, const float* __restrict__ bias, int t,
                                               int lane, uint2 (&av)[KS], float (&bb)[4])
{
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) av[ks] = reinterpret_cast<const uint2*>(wp)[(t * KS + ks) * 64 + lane];
#pragma unroll
    for (int i = 0; i < 4; ++i) bb[i] = bias ? bias[t * 16 + 4 * (lane >> 4) + i] : 0.f;
}

template <int CIN, int COUT, int S, int IX, int IP, int OY, int OX, int OP>
__device__ __forceinline__ void fused_layer(const uint16_t* in_l, uint16_t* out_l, const uint2 (&av)[(9 * CIN + 15) / 16],
                                            const float (&bb)[4], int gy0, int gx0, int Ho, int Wo, int w, int lane)
{
    constexpr int K = 9 * CIN, KS = (K + 15) / 16, MT = (COUT + 15) / 16;
    static_assert(MT == 2, "two 16-channel groups: wave w keeps group w % 2");
    constexpr int NP = OY * OX, PT = (NP + 15) / 16;
    const int g = lane >> 4;
    const int t = w & 1;
    for (int pt = w >> 1; pt < PT; pt += FNW / 2) {
        const int p = pt * 16 + (lane & 15);
        const bool valid = p < NP;
        const int ly = valid ? p / OX : 0, lx = valid ? p - (p / OX) * OX : 0;
        uint2 bv[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k0 = ks * 16 + 4 * g;
            bv[ks] = make_uint2(0u, 0u);
            if (k0 < K) {
                const int tap = k0 / CIN, c = k0 - tap * CIN;
                const int iy = S * ly + tap / 3, ix = S * lx + tap % 3;
                bv[ks] = *reinterpret_cast<const uint2*>(in_l + (iy * IX + ix) * IP + c);
            }
        }
        v4f32 acc = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) acc = mfma(as_v4(av[ks]), as_v4(bv[ks]), acc);
        if (valid) {
            const int o0 = t * 16 + 4 * g;
            const int gy = gy0 + ly, gx = gx0 + lx;
            const bool inside = gy >= 0 && gy < Ho && gx >= 0 && gx < Wo;
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = inside ? fmaxf(acc[i] + bb[i], 0.f) : 0.f;
            *reinterpret_cast<uint2*>(out_l + (ly * OX + lx) * OP + o0) = pack4(v[0], v[1], v[2], v[3]);
        }
    }
}

// Copy the rows [r0, r0 + ny) x columns [c0, c0 + nx) of an LDS region
// [.][LX][32] (grid position of local (0, 0): (gy0, gx0)) to the global
// [Ho][Wo][32] map, positions inside the grid only.
__device__ __forceinline__ void fused_store_acts(const uint16_t* l, int LX, int LP, int r0, int c0, int ny, int nx, int gy0,
                                                 int gx0, uint16_t* __restrict__ g, int Ho, int Wo, int tid)
{
    for (int e = tid; e < ny * nx * 4; e += FNW * 64) {
        const int q = e & 3, pix = e >> 2;                   // 8 channels (16 bytes) per element
        const int y = r0 + pix / nx, x = c0 + pix % nx;
        const int gy = gy0 + y, gx = gx0 + x;
        if (gy < 0 || gy >= Ho || gx < 0 || gx >= Wo) continue;
        const uint2* sp = reinterpret_cast<const uint2*>(l + (y * LX + x) * LP + 8 * q);   // 8-byte aligned
        const uint2 lo = sp[0], hi = sp[1];
        *reinterpret_cast<uint4*>(g + ((size_t)gy * Wo + gx) * 32 + 8 * q) = make_uint4(lo.x, lo.y, hi.x, hi.y);
    }
}

// Eight waves per workgroup, at most two workgroups per CU (four waves per
// SIMD): registers up to that occupancy keep every A operand of a layer in
// VGPRs.
template <bool ACTS>
__global__ __launch_bounds__(FNW * 64) __attribute__((amdgpu_waves_per_eu(1, 4))) void cnn_fused_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wf,
                                                        const float* __restrict__ params, float* __restrict__ out,
                                                        int Hq, int Wq, int H1, int W1, int H2, int W2, int tiles_x,
                                                        int tiles_img, int off1, int off2, int off3,
                                                        uint16_t* __restrict__ a0, uint16_t* __restrict__ a1,
                                                        uint16_t* __restrict__ a2)
{
    __shared__ __attribute__((aligned(16))) uint16_t s_in[FIY * FIX * PIN];
    __shared__ __attribute__((aligned(16))) uint16_t s_0[F0Y * F0X * P0];
    __shared__ __attribute__((aligned(16))) uint16_t s_1[F1Y * F1X * P1];
    __shared__ __attribute__((aligned(16))) uint16_t s_2[F2Y * F2X * P2];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    // neighbouring tiles share input rows: contiguous tile ranges per XCD
    const int nwg = gridDim.x, xcd = blockIdx.x & 7, kq = blockIdx.x >> 3;
    const int wg = xcd * (nwg >> 3) + min(xcd, nwg & 7) + kq;
    const int img = wg / tiles_img, tt = wg - img * tiles_img;
    const int by0 = (tt / tiles_x) * FTY, bx0 = (tt % tiles_x) * FTX;
    // grid positions of local (0, 0) per layer
    const int y2 = by0 - 1, x2 = bx0 - 1, y1 = by0 - 2, x1 = bx0 - 2;
    const int y0 = 2 * y1 - 1, x0 = 2 * x1 - 1, yi = 2 * y0 - 1, xi = 2 * x0 - 1;

    const int t = w & 1;
    uint2 av0[5];
    float bb0[4];
    fused_operands<5>(wf, params + 2304, t, lane, av0, bb0);
    // pooled input: every load of the thread in flight before the LDS writes
    const uint16_t* src = in + (size_t)img * Hq * Wq * 8;
    constexpr int NIN = (FIY * FIX + FNW * 64 - 1) / (FNW * 64);
    uint4 vin[NIN];
#pragma unroll
    for (int r = 0; r < NIN; ++r) {
        const int e = tid + r * FNW * 64;
        const int y = e / FIX, x = e - (e / FIX) * FIX;
        const int gy = yi + y, gx = xi + x;
        vin[r] = make_uint4(0u, 0u, 0u, 0u);
        if (e < FIY * FIX && gy >= 0 && gy < Hq && gx >= 0 && gx < Wq)
            vin[r] = *reinterpret_cast<const uint4*>(src + ((size_t)gy * Wq + gx) * 8);
    }
#pragma unroll
    for (int r = 0; r < NIN; ++r) {
        const int e = tid + r * FNW * 64;
        if (e < FIY * FIX) {
            *reinterpret_cast<uint2*>(s_in + e * PIN) = make_uint2(vin[r].x, vin[r].y);
            *reinterpret_cast<uint2*>(s_in + e * PIN + 4) = make_uint2(vin[r].z, vin[r].w);
        }
    }
    __syncthreads();
    fused_layer<8, 32, 2, FIX, PIN, F0Y, F0X, P0>(s_in, s_0, av0, bb0, y0, x0, H1, W1, w, lane);
    uint2 av1[18];
    float bb1[4];
    fused_operands<18>(wf + off1, params + 11552, t, lane, av1, bb1);
    __syncthreads();
    fused_layer<32, 32, 2, F0X, P0, F1Y, F1X, P1>(s_0, s_1, av1, bb1, y1, x1, H2, W2, w, lane);
    uint2 av2[18];
    float bb2[4];
    fused_operands<18>(wf + off2, params + 20800, t, lane, av2, bb2);
    __syncthreads();
    fused_layer<32, 32, 1, F1X, P1, F2Y, F2X, P2>(s_1, s_2, av2, bb2, y2, x2, H2, W2, w, lane);
    // layer 3's A operands (one 16-channel group, wave 0), before the barrier
    uint2 av3[18];
    float bb3[4];
    if (w == 0) fused_operands<18>(wf + off3, nullptr, 0, lane, av3, bb3);
    __syncthreads();
    if (ACTS) {
        uint16_t* g0 = a0 + (size_t)img * H1 * W1 * 32;
        uint16_t* g1 = a1 + (size_t)img * H2 * W2 * 32;
        uint16_t* g2 = a2 + (size_t)img * H2 * W2 * 32;
        fused_store_acts(s_0, F0X, P0, 2 * by0 - y0, 2 * bx0 - x0, 2 * FTY, 2 * FTX, y0, x0, g0, H1, W1, tid);
        fused_store_acts(s_1, F1X, P1, by0 - y1, bx0 - x1, FTY, FTX, y1, x1, g1, H2, W2, tid);
        fused_store_acts(s_2, F2X, P2, by0 - y2, bx0 - x2, FTY, FTX, y2, x2, g2, H2, W2, tid);
    }
    // layer 3 (32 -> 3, no ReLU, float32 [3][H2][W2]): one 16-pixel tile, wave 0
    if (w != 0) return;
    constexpr int K = 9 * 32, KS = K / 16;
    const int g = lane >> 4;
    const int p = lane & 15;
    const bool valid = p < FTY * FTX;
    const int ly = valid ? p / FTX : 0, lx = valid ? p % FTX : 0;
    uint2 bv[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k0 = ks * 16 + 4 * g;
        const int tap = k0 / 32, c = k0 - tap * 32;
        bv[ks] = *reinterpret_cast<const uint2*>(s_2 + ((ly + tap / 3) * F2X + lx + tap % 3) * P2 + c);
    }
    v4f32 acc = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) acc = mfma(as_v4(av3[ks]), as_v4(bv[ks]), acc);
    const int by = by0 + ly, bx = bx0 + lx;
    if (!valid || by >= H2 || bx >= W2) return;
    const float* b3 = params + 21696;
    float* o = out + (size_t)img * 3 * H2 * W2 + (size_t)by * W2 + bx;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (4 * g + i < 3) o[(size_t)(4 * g + i) * H2 * W2] = acc[i] + b3[4 * g + i];
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

// grads (flat layout: W[o][c][ky][kx] then b[o]) = fixed-order sum of the nwg
// per-workgroup partials of every weight and bias gradient: 64 outputs per
// workgroup; wave q sums partials q, q + 4, q + 8, ...
// in ascending order (independent loads, many in flight), then wave 0 adds
// the four sums in wave order.  The order never depends on timing, so the
// same inputs give the same bits.
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float* __restrict__ partial, int nwg, int cin,
                                                           int cout, int off_w, int off_b, float* __restrict__ grads)
{
    __shared__ float part[3][64];
    const int K = 9 * cin, nw = cout * K, m = nw + cout;
    const int j = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + j;
    float s = 0.f;
    if (e < m) {
        const float* src = e < nw ? partial + e : partial + (size_t)nwg * nw + (e - nw);
        const size_t stride = e < nw ? (size_t)nw : (size_t)cout;
#pragma unroll 8
        for (int w = q; w < nwg; w += 4) s += src[(size_t)w * stride];
    }
    if (q > 0) part[q - 1][j] = s;
    __syncthreads();
    if (q != 0 || e >= m) return;
    s = s + part[0][j];
    s = s + part[1][j];
    s = s + part[2][j];
    if (e < nw) {
        const int o = e / K, k = e - o * K;
        const int tap = k / cin, c = k - tap * cin;
        grads[off_w + (o * cin + c) * 9 + tap] = s;
    } else {
        grads[off_b + (e - nw)] = s;
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

hipError_t launch_cnn_fused(const uint16_t* in, const uint16_t* wf, const float* params, float* out, int n, int Hq,
                            int Wq, uint16_t* a0, uint16_t* a1, uint16_t* a2, hipStream_t st)
{
    const int H1 = (Hq + 1) / 2, W1 = (Wq + 1) / 2, H2 = (H1 + 1) / 2, W2 = (W1 + 1) / 2;
    const int tiles_x = div_up(W2, FTX), tiles_img = div_up(H2, FTY) * tiles_x;
    const long long nwg = (long long)n * tiles_img;
    if (nwg <= 0 || nwg > 0x7fffffffLL) return hipErrorInvalidValue;
    const int off1 = packed_fwd(kCin[0], kCout[0]), off2 = off1 + packed_fwd(kCin[1], kCout[1]);
    const int off3 = off2 + packed_fwd(kCin[2], kCout[2]);
    if (a0)
        hipLaunchKernelGGL(cnn_fused_kernel<true>, dim3((unsigned)nwg), dim3(FNW * 64), 0, st, in, wf, params, out, Hq, Wq,
                           H1, W1, H2, W2, tiles_x, tiles_img, off1, off2, off3, a0, a1, a2);
    else
        hipLaunchKernelGGL(cnn_fused_kernel<false>, dim3((unsigned)nwg), dim3(FNW * 64), 0, st, in, wf, params, out, Hq,
                           Wq, H1, W1, H2, W2, tiles_x, tiles_img, off1, off2, off3, a0, a1, a2);
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
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(div_up(m, 64)), dim3(256), 0, st, partial, nwg, cin[l], cout[l],
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
