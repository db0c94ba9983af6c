// Perception residual network (PRNet, paper Sec. 3.3) on gfx950: the layer
// kernels of its forward and backward passes and its weighted BerHu loss.
//
// Activations are bfloat16, channels last ([pixel][C], pixel = (n, y, x)).
// Features at the network's boundary (z_pred, z_target, the residual and the
// corrected output) are [n][C][Hf][Wf], as the warp writes them.
//
// 1x1 convolutions are GEMMs on v_mfma_f32_16x16x16_bf16: out[p][o] =
// sum_k W[o][k] x[p][k], with m = output channel, n = pixel, k = input
// channel.  A workgroup stages the inputs of 64 pixels in LDS (converting
// float32 or channels-first sources on the way, concatenating two sources
// along k) and each wave produces 16 pixels for every output channel, with
// bias, ReLU6, an added tensor and a ReLU6-derivative mask fused into the
// store.  The same kernel computes input gradients (m = input channel, k =
// output channel, from a transposed packing of W).  Weight gradients reduce
// over pixels (k = pixel) from LDS tiles stored channel-major, into
// per-workgroup partials that a second kernel sums in workgroup order.
//
// Depthwise 3x3 convolutions, their input gradients and the loss are
// bandwidth-bound elementwise stencils on the vector ALUs: one thread per
// pixel and four channels (8-byte accesses, consecutive threads on
// consecutive channels).  Depthwise weight gradients accumulate per thread
// and reduce in a fixed order in LDS.  Nothing uses float atomics, so every
// result is bit-reproducible.
#include "bf16.h"
#include "internal.h"

namespace me {
namespace {

constexpr int kPx = 64;       // pixels per GEMM workgroup
constexpr int kNG = 8;        // output-channel tiles per accumulation pass
constexpr int kTPW = 16;      // weight-gradient tiles per wave
constexpr int kLdp = kPx + 8; // LDS row length (bfloat16) of channel-major tiles

inline int div_up(int a, int b) { return (a + b - 1) / b; }

// 4 consecutive channels c..c+3 of pixel p.
__device__ __forceinline__ float4 load4(const PwTensor& t, int p, int c, int HW)
{
    if (!t.chw) {
        const size_t idx = (size_t)p * t.C + c;
        if (t.f32) return *reinterpret_cast<const float4*>(static_cast<const float*>(t.p) + idx);
        return unpack4(*reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(t.p) + idx));
    }
    const int img = p / HW, hw = p - img * HW;
    const size_t base = ((size_t)img * t.C + c) * HW + hw;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const size_t idx = base + (size_t)i * HW;
        v[i] = t.f32 ? static_cast<const float*>(t.p)[idx] : bf2f(static_cast<const uint16_t*>(t.p)[idx]);
    }
    return make_float4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ void store4(void* out, int chw, int f32, int C, int HW, int p, int c, float4 v)
{
    if (!chw) {
        const size_t idx = (size_t)p * C + c;
        if (f32) *reinterpret_cast<float4*>(static_cast<float*>(out) + idx) = v;
        else *reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + idx) = pack4(v.x, v.y, v.z, v.w);
        return;
    }
    const int img = p / HW, hw = p - img * HW;
    const size_t base = ((size_t)img * C + c) * HW + hw;
    const float a[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const size_t idx = base + (size_t)i * HW;
        if (f32) static_cast<float*>(out)[idx] = a[i];
        else static_cast<uint16_t*>(out)[idx] = f2bf(a[i]);
    }
}

__device__ __forceinline__ float relu6f(float v) { return fminf(fmaxf(v, 0.f), 6.f); }
__device__ __forceinline__ float keep(float m) { return (m > 0.f && m < 6.f) ? 1.f : 0.f; }

// Pixels [p0, p0 + 64) of t into LDS rows (pixel-major: lds[px * ldk + koff + c]).
__device__ void stage_rows(const PwTensor& t, int koff, int p0, int P, int HW, uint16_t* lds, int ldk)
{
    if (!t.chw) {
        const int c4n = t.C >> 2;
        for (int e = threadIdx.x; e < kPx * c4n; e += blockDim.x) {
            const int px = e / c4n, c4 = e - px * c4n, p = p0 + px;
            uint2 v = make_uint2(0u, 0u);
            if (p < P) {
                if (t.f32) {
                    const float4 f = reinterpret_cast<const float4*>(t.p)[(size_t)p * c4n + c4];
                    v = pack4(f.x, f.y, f.z, f.w);
                } else {
                    v = reinterpret_cast<const uint2*>(t.p)[(size_t)p * c4n + c4];
                }
            }
            *reinterpret_cast<uint2*>(lds + px * ldk + koff + 4 * c4) = v;
        }
    } else {
        for (int e = threadIdx.x; e < kPx * t.C; e += blockDim.x) {
            const int c = e / kPx, px = e - c * kPx, p = p0 + px;
            uint16_t v = 0;
            if (p < P) {
                const int img = p / HW, hw = p - img * HW;
                const size_t idx = ((size_t)img * t.C + c) * HW + hw;
                v = t.f32 ? f2bf(static_cast<const float*>(t.p)[idx]) : static_cast<const uint16_t*>(t.p)[idx];
            }
            lds[px * ldk + koff + c] = v;
        }
    }
}

// Pixels [p0, p1) of t into LDS columns (channel-major: lds[(koff + c) * kLdp + px]); pixels past p1 read 0.
__device__ void stage_cols(const PwTensor& t, int koff, int p0, int p1, int HW, uint16_t* lds)
{
    if (!t.chw) {
        const int c4n = t.C >> 2;
        for (int e = threadIdx.x; e < kPx * c4n; e += blockDim.x) {
            const int px = e / c4n, c4 = e - px * c4n, p = p0 + px;
            float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
            uint2 v = make_uint2(0u, 0u);
            if (p < p1) {
                if (t.f32) {
                    f = reinterpret_cast<const float4*>(t.p)[(size_t)p * c4n + c4];
                    v = pack4(f.x, f.y, f.z, f.w);
                } else {
                    v = reinterpret_cast<const uint2*>(t.p)[(size_t)p * c4n + c4];
                }
            }
            uint16_t* d = lds + (koff + 4 * c4) * kLdp + px;
            d[0] = (uint16_t)(v.x & 0xffff);
            d[kLdp] = (uint16_t)(v.x >> 16);
            d[2 * kLdp] = (uint16_t)(v.y & 0xffff);
            d[3 * kLdp] = (uint16_t)(v.y >> 16);
        }
    } else {
        for (int e = threadIdx.x; e < kPx * t.C; e += blockDim.x) {
            const int c = e / kPx, px = e - c * kPx, p = p0 + px;
            uint16_t v = 0;
            if (p < p1) {
                const int img = p / HW, hw = p - img * HW;
                const size_t idx = ((size_t)img * t.C + c) * HW + hw;
                v = t.f32 ? f2bf(static_cast<const float*>(t.p)[idx]) : static_cast<const uint16_t*>(t.p)[idx];
            }
            lds[(koff + c) * kLdp + px] = v;
        }
    }
}

// ------------------------------------------------------------ 1x1 GEMM --

__global__ __launch_bounds__(256) void pw_kernel(PwArgs a)
{
    extern __shared__ uint16_t lds[];
    const int K = a.KS * 16, ldk = K + 8;
    const int p0 = blockIdx.x * kPx;
    stage_rows(a.x, 0, p0, a.P, a.HW, lds, ldk);
    int kc = a.x.C;
    if (a.x2.p) {
        stage_rows(a.x2, kc, p0, a.P, a.HW, lds, ldk);
        kc += a.x2.C;
    }
    for (int e = threadIdx.x; e < kPx * (K - kc); e += blockDim.x) {
        const int px = e / (K - kc), k = kc + e - px * (K - kc);
        lds[px * ldk + k] = 0;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
    const uint16_t* brow = lds + (16 * w + n) * ldk + 4 * g;
    const uint2* wp = reinterpret_cast<const uint2*>(a.w);
    const int MT = (a.M + 15) >> 4;
    const int p = p0 + 16 * w + n;
    for (int mt0 = 0; mt0 < MT; mt0 += kNG) {
        v4f32 acc[kNG];
#pragma unroll
        for (int t = 0; t < kNG; ++t) acc[t] = (v4f32){0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < a.KS; ++ks) {
            const v4i16 b = as_v4(*reinterpret_cast<const uint2*>(brow + ks * 16));
#pragma unroll
            for (int t = 0; t < kNG; ++t)
                if (mt0 + t < MT) acc[t] = mfma(as_v4(wp[((size_t)(mt0 + t) * a.KS + ks) * 64 + lane]), b, acc[t]);
        }
        if (p < a.P) {
#pragma unroll
            for (int t = 0; t < kNG; ++t) {
                if (mt0 + t >= MT) break;
                const int o = (mt0 + t) * 16 + 4 * g;
                if (o >= a.M) break;
                float v[4] = {acc[t][0], acc[t][1], acc[t][2], acc[t][3]};
                if (a.bias) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] += a.bias[o + i];
                }
                if (a.relu6) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = relu6f(v[i]);
                }
                if (a.add.p) {
                    const float4 d = load4(a.add, p, o, a.HW);
                    v[0] += d.x;
                    v[1] += d.y;
                    v[2] += d.z;
                    v[3] += d.w;
                }
                if (a.mask) {
                    const float4 m = unpack4(*reinterpret_cast<const uint2*>(a.mask + (size_t)p * a.M + o));
                    v[0] *= keep(m.x);
                    v[1] *= keep(m.y);
                    v[2] *= keep(m.z);
                    v[3] *= keep(m.w);
                }
                store4(a.out, a.out_chw, a.out_f32, a.M, a.HW, p, o, make_float4(v[0], v[1], v[2], v[3]));
            }
        }
    }
}

// A operand packing: out[(mt * KS + ks) * 64 + L] holds A[m = mt*16 + L%16][k = ks*16 + 4(L/16) + i],
// A[m][k] = trans ? w[k * ld + m0 + m] : w[m * ld + k], zero outside m < Mv, k < Kv.
__global__ void pw_pack_kernel(const float* __restrict__ w, int ld, int m0, int trans, int Mv, int Kv, int MT, int KS,
                               uint2* __restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MT * KS * 64) return;
    const int L = e & 63, q = e >> 6, ks = q % KS, mt = q / KS;
    const int m = mt * 16 + (L & 15), kb = ks * 16 + 4 * (L >> 4);
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = kb + i;
        v[i] = (m < Mv && k < Kv) ? (trans ? w[(size_t)k * ld + m0 + m] : w[(size_t)m * ld + k]) : 0.f;
    }
    out[e] = pack4(v[0], v[1], v[2], v[3]);
}

// ---------------------------------------------------- 1x1 weight gradient --

// grid (nwg, tile groups).  Workgroup x reduces pixels [x*chunk, (x+1)*chunk)
// for the (mt, nt) tiles of its group; tile (mt, nt) = dW[o = mt*16..][c = nt*16..].
__global__ __launch_bounds__(256) void pw_wgrad_kernel(PwGradArgs a)
{
    extern __shared__ uint16_t lds[];
    const int MP = (a.cout + 15) & ~15, NP = (a.cin + 15) & ~15;
    uint16_t* dyT = lds;
    uint16_t* xT = lds + MP * kLdp;
    const int MT = MP >> 4, NT = NP >> 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
    const int t0 = blockIdx.y * 4 * kTPW, t1 = min(MT * NT, t0 + 4 * kTPW);
    const int pb = blockIdx.x * a.chunk, pe = min(a.P, pb + a.chunk);
    const bool do_bias = blockIdx.y == 0;

    v4f32 acc[kTPW];
#pragma unroll
    for (int j = 0; j < kTPW; ++j) acc[j] = (v4f32){0.f, 0.f, 0.f, 0.f};
    float bacc[4] = {0.f, 0.f, 0.f, 0.f};      // output channels threadIdx.x + 256 j

    for (int pc = pb; pc < pe; pc += kPx) {
        __syncthreads();
        stage_cols(a.dy, 0, pc, pe, a.HW, dyT);
        for (int e = threadIdx.x; e < (MP - a.cout) * kLdp; e += blockDim.x) dyT[a.cout * kLdp + e] = 0;
        stage_cols(a.x, 0, pc, pe, a.HW, xT);
        if (a.x2.p) stage_cols(a.x2, a.x.C, pc, pe, a.HW, xT);
        for (int e = threadIdx.x; e < (NP - a.cin) * kLdp; e += blockDim.x) xT[a.cin * kLdp + e] = 0;
        __syncthreads();
        if (do_bias) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = threadIdx.x + 256 * j;
                if (o < a.cout) {
                    const uint16_t* r = dyT + o * kLdp;
                    for (int px = 0; px < kPx; ++px) bacc[j] += bf2f(r[px]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kTPW; ++j) {
            const int tau = t0 + w + 4 * j;
            if (tau < t1) {
                const int mt = tau / NT, nt = tau - mt * NT;
                const uint16_t* ar = dyT + (mt * 16 + n) * kLdp + 4 * g;
                const uint16_t* br = xT + (nt * 16 + n) * kLdp + 4 * g;
#pragma unroll
                for (int ks = 0; ks < kPx / 16; ++ks)
                    acc[j] = mfma(as_v4(*reinterpret_cast<const uint2*>(ar + ks * 16)),
                                  as_v4(*reinterpret_cast<const uint2*>(br + ks * 16)), acc[j]);
            }
        }
    }
    float* pw = a.partial + (size_t)blockIdx.x * a.cout * a.cin;
#pragma unroll
    for (int j = 0; j < kTPW; ++j) {
        const int tau = t0 + w + 4 * j;
        if (tau >= t1) continue;
        const int mt = tau / NT, nt = tau - mt * NT;
        const int c = nt * 16 + n;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = mt * 16 + 4 * g + i;
            if (o < a.cout && c < a.cin) pw[(size_t)o * a.cin + c] = acc[j][i];
        }
    }
    if (do_bias) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = threadIdx.x + 256 * j;
            if (o < a.cout) a.partial[(size_t)gridDim.x * a.cout * a.cin + (size_t)blockIdx.x * a.cout + o] = bacc[j];
        }
    }
}

// grads[off_w + o*cin + c] and grads[off_b + o]: sums of the partials in workgroup order.
__global__ void pw_wgrad_reduce_kernel(const float* __restrict__ partial, int nwg, int cin, int cout,
                                       float* __restrict__ gw, float* __restrict__ gb)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * cin;
    if (e < nw) {
        float s = 0.f;
        for (int x = 0; x < nwg; ++x) s += partial[(size_t)x * nw + e];
        gw[e] = s;
    } else if (e < nw + cout) {
        const int o = e - nw;
        float s = 0.f;
        for (int x = 0; x < nwg; ++x) s += partial[(size_t)nwg * nw + (size_t)x * cout + o];
        gb[o] = s;
    }
}

// ------------------------------------------------------------ depthwise --

template <int S>
__global__ __launch_bounds__(256) void dw_fwd_kernel(const uint16_t* __restrict__ x, const float* __restrict__ w,
                                                     const float* __restrict__ b, uint16_t* __restrict__ y, int n, int H,
                                                     int W, int C, int Ho, int Wo, int relu6)
{
    const int c4n = C >> 2;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * Ho * Wo * c4n) return;
    const int c4 = (int)(e % c4n);
    size_t q = e / c4n;
    const int ox = (int)(q % Wo);
    q /= Wo;
    const int oy = (int)(q % Ho), img = (int)(q / Ho);
    const int c = 4 * c4;
    float acc[4] = {b[c], b[c + 1], b[c + 2], b[c + 3]};
    const uint2* xs = reinterpret_cast<const uint2*>(x) + (size_t)img * H * W * c4n + c4;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
        const int iy = S * oy + ky - 1;
        if (iy < 0 || iy >= H) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            const int ix = S * ox + kx - 1;
            if (ix < 0 || ix >= W) continue;
            const float4 v = unpack4(xs[((size_t)iy * W + ix) * c4n]);
            const int tap = 3 * ky + kx;
            acc[0] += w[c * 9 + tap] * v.x;
            acc[1] += w[(c + 1) * 9 + tap] * v.y;
            acc[2] += w[(c + 2) * 9 + tap] * v.z;
            acc[3] += w[(c + 3) * 9 + tap] * v.w;
        }
    }
    if (relu6) {
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = relu6f(acc[i]);
    }
    reinterpret_cast<uint2*>(y)[e] = pack4(acc[0], acc[1], acc[2], acc[3]);
}

// dx[n][y][x][c] = sum over taps whose output position exists of W[c][tap] dy, times the
// ReLU6 derivative of mask (the stored input activation) when mask is given.
template <int S>
__global__ __launch_bounds__(256) void dw_dgrad_kernel(const uint16_t* __restrict__ dy, const float* __restrict__ w,
                                                       const uint16_t* __restrict__ mask, uint16_t* __restrict__ dx,
                                                       int n, int H, int W, int C, int Ho, int Wo)
{
    const int c4n = C >> 2;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * H * W * c4n) return;
    const int c4 = (int)(e % c4n);
    size_t q = e / c4n;
    const int ix = (int)(q % W);
    q /= W;
    const int iy = (int)(q % H), img = (int)(q / H);
    const int c = 4 * c4;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    const uint2* ds = reinterpret_cast<const uint2*>(dy) + (size_t)img * Ho * Wo * c4n + c4;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
        const int ty = iy + 1 - ky;
        if (ty < 0 || ty % S) continue;
        const int oy = ty / S;
        if (oy >= Ho) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            const int tx = ix + 1 - kx;
            if (tx < 0 || tx % S) continue;
            const int ox = tx / S;
            if (ox >= Wo) continue;
            const float4 d = unpack4(ds[((size_t)oy * Wo + ox) * c4n]);
            const int tap = 3 * ky + kx;
            acc[0] += w[c * 9 + tap] * d.x;
            acc[1] += w[(c + 1) * 9 + tap] * d.y;
            acc[2] += w[(c + 2) * 9 + tap] * d.z;
            acc[3] += w[(c + 3) * 9 + tap] * d.w;
        }
    }
    if (mask) {
        const float4 m = unpack4(reinterpret_cast<const uint2*>(mask)[e]);
        acc[0] *= keep(m.x);
        acc[1] *= keep(m.y);
        acc[2] *= keep(m.z);
        acc[3] *= keep(m.w);
    }
    reinterpret_cast<uint2*>(dx)[e] = pack4(acc[0], acc[1], acc[2], acc[3]);
}

// Partial weight and bias gradients of one workgroup's output pixels:
// partial[wg][c][tap] (tap 9 = bias).  Threads are (channel group, lane of
// the group); each lane accumulates every tpg-th pixel, and the lanes of a
// group are summed in lane order.
template <int S>
__global__ __launch_bounds__(256) void dw_wgrad_kernel(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy,
                                                       float* __restrict__ partial, int n, int H, int W, int C, int Ho,
                                                       int Wo, int chunk)
{
    __shared__ float red[256 * 41];
    const int G = C >> 2, tpg = blockDim.x / G;
    const int grp = threadIdx.x % G, sub = threadIdx.x / G;
    const int P = n * Ho * Wo;
    const int pb = blockIdx.x * chunk, pe = min(P, pb + chunk);
    float acc[10][4];
#pragma unroll
    for (int t = 0; t < 10; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[t][i] = 0.f;
    if (sub < tpg) {
        const uint2* xs = reinterpret_cast<const uint2*>(x) + grp;
        const uint2* ds = reinterpret_cast<const uint2*>(dy) + grp;
        for (int q = pb + sub; q < pe; q += tpg) {
            const int img = q / (Ho * Wo), rem = q - img * Ho * Wo;
            const int oy = rem / Wo, ox = rem - oy * Wo;
            const float4 d = unpack4(ds[(size_t)q * G]);
            acc[9][0] += d.x;
            acc[9][1] += d.y;
            acc[9][2] += d.z;
            acc[9][3] += d.w;
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                const int iy = S * oy + ky - 1;
                if (iy < 0 || iy >= H) continue;
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int ix = S * ox + kx - 1;
                    if (ix < 0 || ix >= W) continue;
                    const float4 v = unpack4(xs[(((size_t)img * H + iy) * W + ix) * G]);
                    const int tap = 3 * ky + kx;
                    acc[tap][0] += d.x * v.x;
                    acc[tap][1] += d.y * v.y;
                    acc[tap][2] += d.z * v.z;
                    acc[tap][3] += d.w * v.w;
                }
            }
        }
    }
    float* r = red + threadIdx.x * 41;
#pragma unroll
    for (int t = 0; t < 10; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) r[t * 4 + i] = acc[t][i];
    __syncthreads();
    for (int e = threadIdx.x; e < G * 40; e += blockDim.x) {
        const int gg = e / 40, j = e - gg * 40;
        float s = 0.f;
        for (int k = 0; k < tpg; ++k) s += red[(k * G + gg) * 41 + j];
        const int tap = j >> 2, i = j & 3;
        partial[((size_t)blockIdx.x * C + 4 * gg + i) * 10 + tap] = s;
    }
}

__global__ void dw_wgrad_reduce_kernel(const float* __restrict__ partial, int nwg, int C, float* __restrict__ gw,
                                       float* __restrict__ gb)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C * 10) return;
    const int c = e / 10, tap = e - c * 10;
    float s = 0.f;
    for (int x = 0; x < nwg; ++x) s += partial[((size_t)x * C + c) * 10 + tap];
    if (tap < 9) gw[c * 9 + tap] = s;
    else gb[c] = s;
}

// ---------------------------------------------------------------- input --

// out[n][y][x][c] = (mosaic sample (2y + (c>>1), 2x + (c&1)) - 2048) / 1024, rounded.
__global__ void planes_kernel(const uint16_t* __restrict__ m, int64_t pitch, int64_t img_stride, int n, int Hp, int Wp,
                              uint16_t* __restrict__ out)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * Hp * Wp) return;
    const int x = (int)(e % Wp);
    const size_t q = e / Wp;
    const int y = (int)(q % Hp), img = (int)(q / Hp);
    const uint16_t* r = m + img * img_stride + (int64_t)(2 * y) * pitch + 2 * x;
    const float k = 1.f / 1024.f;
    reinterpret_cast<uint2*>(out)[e] = pack4(((float)r[0] - 2048.f) * k, ((float)r[1] - 2048.f) * k,
                                             ((float)r[pitch] - 2048.f) * k, ((float)r[pitch + 1] - 2048.f) * k);
}

// ----------------------------------------------------------------- loss --

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Per position p: s = sum_c |t|, t = z_target - z_pred; bad = tau >= 0 and s / C > tau.
// Counts bad positions and takes max |r - t| (order-free, so exact).
__global__ __launch_bounds__(256) void prloss_stats_kernel(const float* __restrict__ r, const float* __restrict__ zp,
                                                           const float* __restrict__ zt, int n, int C, int HW,
                                                           float tau, int32_t* __restrict__ nbad,
                                                           uint32_t* __restrict__ maxbits)
{
    __shared__ float wm[4];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    float mx = 0.f;
    int bad = 0;
    if (p < n * HW) {
        const int img = p / HW, hw = p - img * HW;
        const size_t base = (size_t)img * C * HW + hw;
        float s = 0.f;
        for (int c = 0; c < C; ++c) {
            const size_t i = base + (size_t)c * HW;
            const float t = zt[i] - zp[i];
            s += fabsf(t);
            mx = fmaxf(mx, fabsf(r[i] - t));
        }
        bad = tau >= 0.f && s / (float)C > tau;
    }
    const int cnt = __syncthreads_count(bad);
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
        if (cnt) atomicAdd(nbad, cnt);
        atomicMax(maxbits, __float_as_uint(m));
    }
}

// Loss terms and dr = dloss/dr (bfloat16, [n][C][HW]); partial[block] = the block's loss, summed in thread order.
__global__ __launch_bounds__(256) void prloss_grad_kernel(const float* __restrict__ r, const float* __restrict__ zp,
                                                          const float* __restrict__ zt, int n, int C, int HW, float tau,
                                                          const int32_t* __restrict__ nbad,
                                                          const uint32_t* __restrict__ maxbits,
                                                          uint16_t* __restrict__ dr, float* __restrict__ partial)
{
    __shared__ float red[256];
    const int P = n * HW;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const float cth = 0.2f * __uint_as_float(*maxbits);
    const int nb = *nbad, ng = P - nb;
    float lsum = 0.f;
    if (p < P) {
        const int img = p / HW, hw = p - img * HW;
        const size_t base = (size_t)img * C * HW + hw;
        float wpos = 1.f / (float)P;
        if (tau >= 0.f && nb > 0 && ng > 0) {
            float s = 0.f;
            for (int c = 0; c < C; ++c) {
                const size_t i = base + (size_t)c * HW;
                s += fabsf(zt[i] - zp[i]);
            }
            wpos = (s / (float)C > tau) ? 0.5f / (float)nb : 0.5f / (float)ng;
        }
        const float wgt = wpos / (float)C;
        for (int c = 0; c < C; ++c) {
            const size_t i = base + (size_t)c * HW;
            const float x = r[i] - (zt[i] - zp[i]);
            const float a = fabsf(x);
            float ber = 0.f, gr = 0.f;
            if (cth > 0.f) {
                if (a <= cth) {
                    ber = a;
                    gr = x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f);
                } else {
                    ber = (x * x + cth * cth) / (2.f * cth);
                    gr = x / cth;
                }
            }
            lsum += ber;
            dr[i] = f2bf(wgt * gr);
        }
        lsum *= wgt;
    }
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void prloss_sum_kernel(const float* __restrict__ partial, int m, float* __restrict__ loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < m; i += blockDim.x) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0];
}

}  // namespace

// ------------------------------------------------------------ host side --

size_t pw_lds_bytes(int KS) { return (size_t)kPx * (KS * 16 + 8) * sizeof(uint16_t); }

size_t pw_wgrad_lds_bytes(int cin, int cout)
{
    return (size_t)(((cout + 15) & ~15) + ((cin + 15) & ~15)) * kLdp * sizeof(uint16_t);
}

int pw_wgrad_groups(int cin, int cout) { return div_up(div_up(cout, 16) * div_up(cin, 16), 4 * kTPW); }

int wgrad_chunk(int P, int target_wg)
{
    const int c = div_up(div_up(P, target_wg), kPx) * kPx;
    return c > 0 ? c : kPx;
}

// Dynamic LDS beyond 64 KB needs the per-kernel limit raised (gfx950: 160 KB per workgroup).
static hipError_t allow_lds(const void* k, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_pw(const PwArgs& a, hipStream_t st)
{
    if (a.P <= 0) return hipSuccess;
    const size_t lds = pw_lds_bytes(a.KS);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(pw_kernel), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pw_kernel, dim3(div_up(a.P, kPx)), dim3(256), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_pw_pack(const float* w, int ld, int m0, int trans, int Mv, int Kv, int MT, int KS, uint16_t* out,
                          hipStream_t st)
{
    const int n = MT * KS * 64;
    hipLaunchKernelGGL(pw_pack_kernel, dim3(div_up(n, 256)), dim3(256), 0, st, w, ld, m0, trans, Mv, Kv, MT, KS,
                       reinterpret_cast<uint2*>(out));
    return hipGetLastError();
}

hipError_t launch_pw_wgrad(const PwGradArgs& a, float* gw, float* gb, hipStream_t st)
{
    const int nwg = div_up(a.P, a.chunk);
    if (a.P > 0) {
        const size_t lds = pw_wgrad_lds_bytes(a.cin, a.cout);
        hipError_t e = allow_lds(reinterpret_cast<const void*>(pw_wgrad_kernel), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pw_wgrad_kernel, dim3(nwg, pw_wgrad_groups(a.cin, a.cout)), dim3(256), lds, st, a);
    }
    const int m = a.cout * a.cin + a.cout;
    hipLaunchKernelGGL(pw_wgrad_reduce_kernel, dim3(div_up(m, 256)), dim3(256), 0, st, a.partial, a.P > 0 ? nwg : 0,
                       a.cin, a.cout, gw, gb);
    return hipGetLastError();
}

hipError_t launch_dw_fwd(const uint16_t* x, const float* w, const float* b, uint16_t* y, int n, int H, int W, int C,
                         int S, int relu6, hipStream_t st)
{
    const int Ho = (H - 1) / S + 1, Wo = (W - 1) / S + 1;
    const size_t m = (size_t)n * Ho * Wo * (C >> 2);
    if (m == 0) return hipSuccess;
    const dim3 grid((unsigned)((m + 255) / 256));
    if (S == 1) hipLaunchKernelGGL(dw_fwd_kernel<1>, grid, dim3(256), 0, st, x, w, b, y, n, H, W, C, Ho, Wo, relu6);
    else hipLaunchKernelGGL(dw_fwd_kernel<2>, grid, dim3(256), 0, st, x, w, b, y, n, H, W, C, Ho, Wo, relu6);
    return hipGetLastError();
}

hipError_t launch_dw_dgrad(const uint16_t* dy, const float* w, const uint16_t* mask, uint16_t* dx, int n, int H, int W,
                           int C, int S, hipStream_t st)
{
    const int Ho = (H - 1) / S + 1, Wo = (W - 1) / S + 1;
    const size_t m = (size_t)n * H * W * (C >> 2);
    if (m == 0) return hipSuccess;
    const dim3 grid((unsigned)((m + 255) / 256));
    if (S == 1) hipLaunchKernelGGL(dw_dgrad_kernel<1>, grid, dim3(256), 0, st, dy, w, mask, dx, n, H, W, C, Ho, Wo);
    else hipLaunchKernelGGL(dw_dgrad_kernel<2>, grid, dim3(256), 0, st, dy, w, mask, dx, n, H, W, C, Ho, Wo);
    return hipGetLastError();
}

hipError_t launch_dw_wgrad(const uint16_t* x, const uint16_t* dy, float* partial, int nwg, int chunk, float* gw,
                           float* gb, int n, int H, int W, int C, int S, hipStream_t st)
{
    const int Ho = (H - 1) / S + 1, Wo = (W - 1) / S + 1;
    if (nwg > 0) {
        if (S == 1)
            hipLaunchKernelGGL(dw_wgrad_kernel<1>, dim3(nwg), dim3(256), 0, st, x, dy, partial, n, H, W, C, Ho, Wo,
                               chunk);
        else
            hipLaunchKernelGGL(dw_wgrad_kernel<2>, dim3(nwg), dim3(256), 0, st, x, dy, partial, n, H, W, C, Ho, Wo,
                               chunk);
    }
    hipLaunchKernelGGL(dw_wgrad_reduce_kernel, dim3(div_up(C * 10, 256)), dim3(256), 0, st, partial, nwg, C, gw, gb);
    return hipGetLastError();
}

hipError_t launch_planes(const uint16_t* m, int64_t pitch, int64_t img_stride, int n, int Hp, int Wp, uint16_t* out,
                         hipStream_t st)
{
    const size_t e = (size_t)n * Hp * Wp;
    if (e == 0) return hipSuccess;
    hipLaunchKernelGGL(planes_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, m, pitch, img_stride, n, Hp,
                       Wp, out);
    return hipGetLastError();
}

int prloss_blocks(int P) { return div_up(P, 256); }

hipError_t launch_prloss(const float* r, const float* zp, const float* zt, int n, int C, int HW, float tau,
                         int32_t* nbad, uint32_t* maxbits, uint16_t* dr, float* partial, float* loss, hipStream_t st)
{
    const int P = n * HW, nb = prloss_blocks(P);
    hipError_t e = launch_fill_i32(nbad, 1, 0, st);
    if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t*>(maxbits), 1, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prloss_stats_kernel, dim3(nb), dim3(256), 0, st, r, zp, zt, n, C, HW, tau, nbad, maxbits);
    hipLaunchKernelGGL(prloss_grad_kernel, dim3(nb), dim3(256), 0, st, r, zp, zt, n, C, HW, tau, nbad, maxbits, dr,
                       partial);
    hipLaunchKernelGGL(prloss_sum_kernel, dim3(1), dim3(256), 0, st, partial, nb, loss);
    return hipGetLastError();
}

}  // namespace me
