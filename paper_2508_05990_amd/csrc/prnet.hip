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
constexpr int kTPW = 16;      // weight-gradient tiles per wave
constexpr int kLdp = kPx + 4; // LDS row length (bfloat16) of channel-major tiles (8-byte aligned rows)

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
    } else if ((HW & 3) == 0) {
        // channels-first, four pixels per thread (a group never straddles two images):
        // 16 lanes cover a 64-pixel channel row
        for (int e = threadIdx.x; e < (kPx / 4) * t.C; e += blockDim.x) {
            const int c = e >> 4, q = e & 15, p = p0 + 4 * q;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (p < P) {
                const int img = p / HW, hw = p - img * HW;
                const size_t idx = ((size_t)img * t.C + c) * HW + hw;
                if (t.f32) {
                    const float4 f = *reinterpret_cast<const float4*>(static_cast<const float*>(t.p) + idx);
                    v[0] = f.x;
                    v[1] = f.y;
                    v[2] = f.z;
                    v[3] = f.w;
                } else {
                    const float4 f = unpack4(*reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(t.p) + idx));
                    v[0] = f.x;
                    v[1] = f.y;
                    v[2] = f.z;
                    v[3] = f.w;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) lds[(4 * q + i) * ldk + koff + c] = f2bf(v[i]);
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
        // a wave covers 16 channel groups x 4 pixels: 128-byte global segments, and
        // its transposed LDS writes spread over 16 banks (4-way) with the 68-element rows
        const int c4n = t.C >> 2, cb = (c4n + 15) >> 4;
        for (int e = threadIdx.x; e < kPx * cb * 16; e += blockDim.x) {
            const int hi = e >> 4, c4 = (hi % cb) * 16 + (e & 15), px = hi / cb;
            if (c4 >= c4n) continue;
            const int p = p0 + px;
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

// Row length (floats) of a wave's transpose slice: NCT 16-pixel column tiles.
__host__ __device__ constexpr int pw_scld(int nct) { return 16 * nct + 4; }

// Channels-first output through the per-wave LDS transpose: four-pixel groups
// never straddle two images when HW is a multiple of 4.
__host__ __device__ inline bool pw_chw_fast(const PwArgs& a)
{
    return a.out_chw && (a.HW & 3) == 0 && !a.mask && (!a.add.p || a.add.chw);
}

// One workgroup of NW waves per 64-pixel tile (grid-stride over tiles).  Wave
// w owns the output row tiles w % 4, w % 4 + 4, ... (16 channels each) for the
// NCT = 16 / NW column tiles (16 pixels each) of part w / 4 of the tile: it
// loads each A operand (packed weights) once and applies it to its column
// tiles read from LDS.  Eight waves halve each wave's chain for grids of about
// one round; four keep more workgroups per CU on larger grids.
template <int NW>
__global__ __launch_bounds__(NW * 64) void pw_kernel(PwArgs a)
{
    extern __shared__ __align__(16) uint16_t lds[];
    const int K = a.KS * 16, ldk = K + 4;   // rows 8-byte aligned, 18 mod 64 banks apart
    const int MT = (a.M + 15) >> 4;
    uint16_t* xl = lds;
    const uint2* wp = reinterpret_cast<const uint2*>(a.w);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
    constexpr int NCT = 16 / NW, kScLd = pw_scld(NCT);
    const int w = wv & 3, half = wv >> 2;                  // row-tile role, column part
    const int ntiles = (a.P + kPx - 1) / kPx;
    const int kc = a.x.C + (a.x2.p ? a.x2.C : 0);
    const bool chw_fast = pw_chw_fast(a);
    float* sc = reinterpret_cast<float*>(xl + kPx * ldk) + wv * 16 * kScLd;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int p0 = tile * kPx;
        __syncthreads();                                   // the previous tile's reads of xl are done
        stage_rows(a.x, 0, p0, a.P, a.HW, xl, ldk);
        if (a.x2.p) stage_rows(a.x2, a.x.C, p0, a.P, a.HW, xl, ldk);
        for (int e = threadIdx.x; e < kPx * (K - kc); e += blockDim.x) {
            const int px = e / (K - kc), k = kc + e - px * (K - kc);
            xl[px * ldk + k] = 0;
        }
        __syncthreads();

        for (int t = w; t < MT; t += 4) {
            v4f32 acc[NCT];
#pragma unroll
            for (int nt = 0; nt < NCT; ++nt) acc[nt] = (v4f32){0.f, 0.f, 0.f, 0.f};
            for (int ks = 0; ks < a.KS; ++ks) {
                const v4i16 wa = as_v4(wp[((size_t)t * a.KS + ks) * 64 + lane]);
#pragma unroll
                for (int nt = 0; nt < NCT; ++nt)
                    acc[nt] = mfma(wa,
                                   as_v4(*reinterpret_cast<const uint2*>(xl + ((NCT * half + nt) * 16 + n) * ldk + ks * 16 + 4 * g)),
                                   acc[nt]);
            }
            const int o = t * 16 + 4 * g;
            float bias[4] = {0.f, 0.f, 0.f, 0.f};
            if (a.bias && o < a.M) {
#pragma unroll
                for (int i = 0; i < 4; ++i) bias[i] = a.bias[o + i];
            }
            if (chw_fast) {
                // channels-first output: transpose the wave's 16 x 16 NCT tile through its LDS
                // slice so that each lane reads/writes four consecutive pixels of one channel
#pragma unroll
                for (int nt = 0; nt < NCT; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float v = acc[nt][i] + bias[i];
                        sc[(4 * g + i) * kScLd + nt * 16 + n] = a.relu6 ? relu6f(v) : v;
                    }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int r = 0; r < NCT; ++r) {
                    const int idx = lane + 64 * r, ch = idx / (4 * NCT), q4 = idx % (4 * NCT);
                    const int oc = t * 16 + ch, px = p0 + 16 * NCT * half + 4 * q4;
                    if (oc >= a.M || px >= a.P) continue;
                    float4 v = *reinterpret_cast<const float4*>(sc + ch * kScLd + 4 * q4);
                    const int img = px / a.HW, hw = px - img * a.HW;
                    const size_t gi = ((size_t)img * a.M + oc) * a.HW + hw;
                    if (a.add.p) {
                        const float4 d = a.add.f32 ? *reinterpret_cast<const float4*>(static_cast<const float*>(a.add.p) + gi)
                                                   : unpack4(*reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(a.add.p) + gi));
                        v.x += d.x;
                        v.y += d.y;
                        v.z += d.z;
                        v.w += d.w;
                    }
                    if (a.out_f32) {
                        // a float32 channels-first output is the network's result: written once, so
                        // non-temporal stores
                        const v4f32 nv = {v.x, v.y, v.z, v.w};
                        __builtin_nontemporal_store(nv, reinterpret_cast<v4f32*>(static_cast<float*>(a.out) + gi));
                    } else {
                        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(a.out) + gi) = pack4(v.x, v.y, v.z, v.w);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                continue;
            }
            if (o >= a.M) continue;
#pragma unroll
            for (int nt = 0; nt < NCT; ++nt) {
                const int p = p0 + (NCT * half + nt) * 16 + n;
                if (p >= a.P) continue;
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = acc[nt][i] + bias[i];
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
    extern __shared__ __align__(16) uint16_t lds[];
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

// ------------------------------------------------------------ depthwise --

constexpr int kRun = 8;   // outputs along x per thread in the depthwise kernels

__device__ __forceinline__ float4 ld4(const uint2* base, int c4n, int H, int W, int r, int c)
{
    if (r < 0 || r >= H || c < 0 || c >= W) return make_float4(0.f, 0.f, 0.f, 0.f);
    return unpack4(base[((size_t)r * W + c) * c4n]);
}

// Depthwise 3x3, zero padding 1, over runs of RUN outputs along x per thread:
// a sliding 3x3 window of 4-channel vectors (3 loads per output at stride 1,
// 6 at stride 2, instead of 9).  GRAD = false: y = b + sum_tap w[tap] x[S oy +
// ky - 1][S ox + kx - 1], then ReLU6 if relu6.  GRAD = true (stride 1 only):
// the input gradient dx[y][x] = sum_tap w[tap] dy[y + 1 - ky][x + 1 - kx], i.e.
// the same pass over dy with the kernel rotated by 180 degrees, times the
// ReLU6 derivative of mask when mask is given.
template <int S, bool GRAD, int RUN>
__global__ __launch_bounds__(256) void dw_fwd_kernel(const uint16_t* __restrict__ x, const float* __restrict__ w,
                                                     const float* __restrict__ b, const uint16_t* __restrict__ mask,
                                                     uint16_t* __restrict__ y, int n, int H, int W, int C, int Ho,
                                                     int Wo, int relu6)
{
    const int c4n = C >> 2, runs = (Wo + RUN - 1) / RUN;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * Ho * runs * c4n) return;
    const int c4 = (int)(e % c4n);
    size_t q = e / c4n;
    const int run = (int)(q % runs);
    q /= runs;
    const int oy = (int)(q % Ho), img = (int)(q / Ho);
    const int c = 4 * c4;
    float wk[9][4];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) wk[t][i] = w[(c + i) * 9 + (GRAD ? 8 - t : t)];
    float bias[4] = {0.f, 0.f, 0.f, 0.f};
    if (!GRAD) {
#pragma unroll
        for (int i = 0; i < 4; ++i) bias[i] = b[c + i];
    }
    const uint2* xs = reinterpret_cast<const uint2*>(x) + (size_t)img * H * W * c4n + c4;
    const int ox0 = run * RUN;
    float4 win[3][3];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
        const int iy = S * oy + ky - 1;
        win[ky][0] = ld4(xs, c4n, H, W, iy, S * ox0 - 1);
        win[ky][1] = ld4(xs, c4n, H, W, iy, S * ox0);
    }
    uint2* ys = reinterpret_cast<uint2*>(y) + ((size_t)(img * Ho + oy) * Wo) * c4n + c4;
    const uint2* ms = mask ? reinterpret_cast<const uint2*>(mask) + ((size_t)(img * Ho + oy) * Wo) * c4n + c4 : nullptr;
#pragma unroll
    for (int j = 0; j < RUN; ++j) {
        const int ox = ox0 + j;
        if (ox >= Wo) break;
        const int ixr = S * ox + 1;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) win[ky][2] = ld4(xs, c4n, H, W, S * oy + ky - 1, ixr);
        float acc[4] = {bias[0], bias[1], bias[2], bias[3]};
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const float4 v = win[ky][kx];
                const int t = 3 * ky + kx;
                acc[0] += wk[t][0] * v.x;
                acc[1] += wk[t][1] * v.y;
                acc[2] += wk[t][2] * v.z;
                acc[3] += wk[t][3] * v.w;
            }
        if (!GRAD && relu6) {
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = relu6f(acc[i]);
        }
        if (GRAD && ms) {
            const float4 m = unpack4(ms[(size_t)ox * c4n]);
            acc[0] *= keep(m.x);
            acc[1] *= keep(m.y);
            acc[2] *= keep(m.z);
            acc[3] *= keep(m.w);
        }
        ys[(size_t)ox * c4n] = pack4(acc[0], acc[1], acc[2], acc[3]);
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            if (S == 1) {
                win[ky][0] = win[ky][1];
                win[ky][1] = win[ky][2];
            } else {
                win[ky][0] = win[ky][2];
                win[ky][1] = ld4(xs, c4n, H, W, S * oy + ky - 1, ixr + 1);
            }
        }
    }
}

// Input gradient at stride 2: dx[n][y][x][c] = sum over the taps whose output
// position exists of W[c][tap] dy, times the ReLU6 derivative of mask.
__global__ __launch_bounds__(256) void dw_dgrad2_kernel(const uint16_t* __restrict__ dy, const float* __restrict__ w,
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
        if (ty < 0 || (ty & 1)) continue;
        const int oy = ty >> 1;
        if (oy >= Ho) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            const int tx = ix + 1 - kx;
            if (tx < 0 || (tx & 1)) continue;
            const int ox = tx >> 1;
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

// Partial weight and bias gradients: partial[wg][c][tap] (tap 9 = bias) over
// the workgroup's units (image, output row, run of kRun outputs).  Threads are
// (channel group, lane of the group); each lane takes every tpg-th unit with a
// sliding input window, and the lanes of a group are summed in lane order.
template <int S>
__global__ __launch_bounds__(256) void dw_wgrad_kernel(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy,
                                                       float* __restrict__ partial, int n, int H, int W, int C, int Ho,
                                                       int Wo, int chunk)
{
    __shared__ float red[256 * 41];
    const int G = C >> 2, tpg = blockDim.x / G;
    const int grp = threadIdx.x % G, sub = threadIdx.x / G;
    const int runs = (Wo + kRun - 1) / kRun, U = n * Ho * runs;
    const int ub = blockIdx.x * chunk, ue = min(U, ub + chunk);
    float acc[10][4];
#pragma unroll
    for (int t = 0; t < 10; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[t][i] = 0.f;
    if (sub < tpg) {
        for (int u = ub + sub; u < ue; u += tpg) {
            const int run = u % runs, q = u / runs, oy = q % Ho, img = q / Ho;
            const uint2* xs = reinterpret_cast<const uint2*>(x) + (size_t)img * H * W * G + grp;
            const uint2* ds = reinterpret_cast<const uint2*>(dy) + ((size_t)(img * Ho + oy) * Wo) * G + grp;
            const int ox0 = run * kRun;
            float4 win[3][3];
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                const int iy = S * oy + ky - 1;
                win[ky][0] = ld4(xs, G, H, W, iy, S * ox0 - 1);
                win[ky][1] = ld4(xs, G, H, W, iy, S * ox0);
            }
#pragma unroll
            for (int j = 0; j < kRun; ++j) {
                const int ox = ox0 + j;
                if (ox >= Wo) break;
                const int ixr = S * ox + 1;
#pragma unroll
                for (int ky = 0; ky < 3; ++ky) win[ky][2] = ld4(xs, G, H, W, S * oy + ky - 1, ixr);
                const float4 d = unpack4(ds[(size_t)ox * G]);
                acc[9][0] += d.x;
                acc[9][1] += d.y;
                acc[9][2] += d.z;
                acc[9][3] += d.w;
#pragma unroll
                for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                    for (int kx = 0; kx < 3; ++kx) {
                        const float4 v = win[ky][kx];
                        const int t = 3 * ky + kx;
                        acc[t][0] += d.x * v.x;
                        acc[t][1] += d.y * v.y;
                        acc[t][2] += d.z * v.z;
                        acc[t][3] += d.w * v.w;
                    }
#pragma unroll
                for (int ky = 0; ky < 3; ++ky) {
                    if (S == 1) {
                        win[ky][0] = win[ky][1];
                        win[ky][1] = win[ky][2];
                    } else {
                        win[ky][0] = win[ky][2];
                        win[ky][1] = ld4(xs, G, H, W, S * oy + ky - 1, ixr + 1);
                    }
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

// Sums of partial rows in a fixed order: element e (< m) of the output is
// sum over rows x of partial[x * stride + e].  Thread group q (of 4) takes rows
// x = q mod 4 into four running sums by (x / 4) mod 4 (independent loads in
// flight), adds them in order, and the four groups are added in q order.  mode 0: out[e];
// mode 1 (depthwise layout [c][10]): tap < 9 -> gw[c*9 + tap], tap 9 -> gb[c].
__global__ __launch_bounds__(256) void reduce_rows_kernel(const float* __restrict__ partial, int nrows, size_t stride,
                                                          int m, int mode, float* __restrict__ gw,
                                                          float* __restrict__ gb)
{
    __shared__ float red[4][64];
    const int j = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + j;
    float s4[4] = {0.f, 0.f, 0.f, 0.f};
    if (e < m) {
        int x = q;
        for (; x + 12 < nrows; x += 16) {
#pragma unroll
            for (int r = 0; r < 4; ++r) s4[r] += partial[(size_t)(x + 4 * r) * stride + e];
        }
        for (int r = 0; x < nrows; x += 4, ++r) s4[r] += partial[(size_t)x * stride + e];
    }
    red[q][j] = ((s4[0] + s4[1]) + s4[2]) + s4[3];
    __syncthreads();
    if (q != 0 || e >= m) return;
    const float t = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    if (mode == 0) {
        gw[e] = t;
    } else {
        const int c = e / 10, tap = e - c * 10;
        if (tap < 9) gw[c * 9 + tap] = t;
        else gb[c] = t;
    }
}

// ------------------------------------------------- fused residual block --

// One inverted residual block in one pass (inference): h_out = h + Wc v + bc,
// v = ReLU6(dw3x3(u) + bd), u = ReLU6(We h + be), with u and v kept in LDS.
// A workgroup owns an 8 x 8 tile of output pixels.  It stages h over the
// tile and its one-pixel halo (10 x 10 = 100 pixels, padded to 7 MFMA column
// tiles), then walks the expanded channels in chunks of 64: expand the chunk
// for all halo pixels (u = 0 outside the image: the depthwise zero padding),
// depthwise-filter it into v (64 x 64), and fold v into the compression
// accumulators, which stay in registers across chunks.  Rounding points match
// the layer-by-layer path (u, v and h_out are bfloat16).  About 44 KB of LDS
// per workgroup at 64 hidden channels.
constexpr int kIrT = 8, kIrHW = kIrT + 2, kIrHalo = kIrHW * kIrHW, kIrRows = 112;
// Row strides (bfloat16 elements) of the staged h (CH + kIrPadH) and of the u
// and v chunks (kIrLd): multiples of 4 (8-byte lane reads), padded so that the
// sixteen rows of an MFMA operand read spread over the LDS banks.
constexpr int kIrPadH = 4, kIrPadU = 4;
constexpr int kIrChunk = 64, kIrLd = kIrChunk + kIrPadU;
// Eight waves: wave w takes the 16-channel row tile w % 4 of each product and
// the pixel column tiles of half w / 4 (expansion: halo column tiles 0-3 or
// 4-6; compression: output column tiles 0-1 or 2-3).
constexpr int kIrThreads = 512;

template <int CH>
__global__ __launch_bounds__(kIrThreads) void ir_block_kernel(IrArgs a)
{
    extern __shared__ __align__(16) uint16_t lds[];
    const int X = a.x;
    constexpr int ldh = CH + kIrPadH;
    uint16_t* hl = lds;                                   // [112][ldh]      h over tile + halo
    uint16_t* ul = hl + kIrRows * ldh;                     // [112][kIrLd]    u, one chunk
    uint16_t* vl = ul + kIrRows * kIrLd;                   // [64][kIrLd]     v, one chunk
    float* wl = reinterpret_cast<float*>(vl + kIrT * kIrT * kIrLd);   // [X][10] depthwise weights + bias, [X] expansion bias
    const int tiles_x = (a.Wf + kIrT - 1) / kIrT, tiles_y = (a.Hf + kIrT - 1) / kIrT;
    const int img = blockIdx.x / (tiles_x * tiles_y), tr = blockIdx.x - img * tiles_x * tiles_y;
    const int y0 = (tr / tiles_x) * kIrT, x0 = (tr % tiles_x) * kIrT;
    constexpr int c4n = CH >> 2;
    const uint2* hin = reinterpret_cast<const uint2*>(a.h_in) + (size_t)img * a.Hf * a.Wf * c4n;

    // every global read but the packed weights happens here, once; a thread issues
    // all of its halo loads (and groups of its parameter loads) before writing
    // LDS, so their latencies overlap (kIrThreads threads, as launched)
    {
        constexpr int kH = (kIrRows * c4n + kIrThreads - 1) / kIrThreads;
        uint2 hv[kH];
#pragma unroll
        for (int u = 0; u < kH; ++u) {
            const int e = threadIdx.x + kIrThreads * u, hp = e / c4n, c4 = e - hp * c4n;
            hv[u] = make_uint2(0u, 0u);
            if (hp < kIrHalo) {
                const int gy = y0 + hp / kIrHW - 1, gx = x0 + hp % kIrHW - 1;
                if (gy >= 0 && gy < a.Hf && gx >= 0 && gx < a.Wf) hv[u] = hin[((size_t)gy * a.Wf + gx) * c4n + c4];
            }
        }
#pragma unroll
        for (int u = 0; u < kH; ++u) {
            const int e = threadIdx.x + kIrThreads * u, hp = e / c4n, c4 = e - hp * c4n;
            if (hp < kIrRows) *reinterpret_cast<uint2*>(hl + hp * ldh + 4 * c4) = hv[u];
        }
    }
    for (int e0 = threadIdx.x; e0 < X * 11; e0 += 4 * kIrThreads) {
        float pv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + kIrThreads * u, ch = e / 11, t = e - ch * 11;
            pv[u] = 0.f;
            if (e < X * 11) pv[u] = t < 9 ? a.wd[ch * 9 + t] : (t == 9 ? a.bd[ch] : a.be[ch]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + kIrThreads * u, ch = e / 11, t = e - ch * 11;
            if (e < X * 11) wl[t < 10 ? ch * 10 + t : X * 10 + ch] = pv[u];
        }
    }

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
    const int w = wv & 3, half = wv >> 2;                  // row-tile role, column half
    const uint2* we = reinterpret_cast<const uint2*>(a.we);
    const uint2* wc = reinterpret_cast<const uint2*>(a.wc);
    constexpr int KSe = CH >> 4, MTc = CH >> 4, MPW = (MTc + 3) / 4;   // compression row tiles per wave
    const int KSc = X >> 4, nq = X / kIrChunk;
    // Role w owns expansion row tile w of every chunk (16 of its 64 channels)
    // and compression row tiles w, w + 4, ...: its two waves load only those
    // weights and reuse them across their half's column (pixel) tiles; the next
    // chunk's weights are loaded while the current chunk is computed.
    v4f32 acc2[MPW][2];
#pragma unroll
    for (int j = 0; j < MPW; ++j)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc2[j][nt] = (v4f32){0.f, 0.f, 0.f, 0.f};
    const int c4 = threadIdx.x & 15;                       // channel group of this thread in the depthwise step
    v4i16 wa[KSe], wb[MPW][4];
#pragma unroll
    for (int ks = 0; ks < KSe; ++ks) wa[ks] = as_v4(we[((size_t)w * KSe + ks) * 64 + lane]);
#pragma unroll
    for (int j = 0; j < MPW; ++j)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            wb[j][ks] = w + 4 * j < MTc ? as_v4(wc[((size_t)(w + 4 * j) * KSc + ks) * 64 + lane]) : as_v4(make_uint2(0u, 0u));
    __syncthreads();

#pragma unroll 1
    for (int q = 0; q < nq; ++q) {
        v4i16 wa_n[KSe], wb_n[MPW][4];
        const int qn = q + 1 < nq ? q + 1 : q;
#pragma unroll
        for (int ks = 0; ks < KSe; ++ks) wa_n[ks] = as_v4(we[((size_t)(4 * qn + w) * KSe + ks) * 64 + lane]);
#pragma unroll
        for (int j = 0; j < MPW; ++j)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                wb_n[j][ks] = w + 4 * j < MTc ? as_v4(wc[((size_t)(w + 4 * j) * KSc + 4 * qn + ks) * 64 + lane])
                                              : as_v4(make_uint2(0u, 0u));
        // expansion: channels 64 q + 16 w .. + 15 for the 112 halo rows (the previous
        // chunk's depthwise reads of u finished before its compression barrier)
        const int oe = 16 * w + 4 * g;
        const float* bexp = wl + X * 10 + q * kIrChunk + oe;
        const float be0 = bexp[0], be1 = bexp[1], be2 = bexp[2], be3 = bexp[3];
#pragma unroll
        for (int ntl = 0; ntl < 4; ++ntl) {
            const int nt = 4 * half + ntl;
            if (nt >= kIrRows / 16) break;
            const int hp = nt * 16 + n;
            const int gy = y0 + hp / kIrHW - 1, gx = x0 + hp % kIrHW - 1;
            const bool inside = hp < kIrHalo && gy >= 0 && gy < a.Hf && gx >= 0 && gx < a.Wf;
            const uint16_t* brow = hl + hp * ldh + 4 * g;
            v4f32 acc = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KSe; ++ks) acc = mfma(wa[ks], as_v4(*reinterpret_cast<const uint2*>(brow + ks * 16)), acc);
            *reinterpret_cast<uint2*>(ul + hp * kIrLd + oe) =
                inside ? pack4(relu6f(acc[0] + be0), relu6f(acc[1] + be1), relu6f(acc[2] + be2), relu6f(acc[3] + be3))
                       : make_uint2(0u, 0u);
        }
        __syncthreads();
        // depthwise: 64 pixels x 16 channel groups, 2 per thread
        float wk[40];
#pragma unroll
        for (int i = 0; i < 40; ++i) wk[i] = wl[(q * kIrChunk + 4 * c4) * 10 + i];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int px = (threadIdx.x >> 4) + 32 * j, ty = px >> 3, tx = px & 7;
            float acc[4] = {wk[9], wk[19], wk[29], wk[39]};
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const float4 u =
                        unpack4(*reinterpret_cast<const uint2*>(ul + ((ty + ky) * kIrHW + tx + kx) * kIrLd + 4 * c4));
                    const int t = 3 * ky + kx;
                    acc[0] += wk[t] * u.x;
                    acc[1] += wk[10 + t] * u.y;
                    acc[2] += wk[20 + t] * u.z;
                    acc[3] += wk[30 + t] * u.w;
                }
            *reinterpret_cast<uint2*>(vl + px * kIrLd + 4 * c4) =
                pack4(relu6f(acc[0]), relu6f(acc[1]), relu6f(acc[2]), relu6f(acc[3]));
        }
        __syncthreads();
        // compression: row tiles w + 4 j over this half's two column tiles (32 pixels)
#pragma unroll
        for (int ntl = 0; ntl < 2; ++ntl) {
            const uint16_t* brow = vl + ((2 * half + ntl) * 16 + n) * kIrLd + 4 * g;
#pragma unroll
            for (int ks = 0; ks < kIrChunk / 16; ++ks) {
                const v4i16 b = as_v4(*reinterpret_cast<const uint2*>(brow + ks * 16));
#pragma unroll
                for (int j = 0; j < MPW; ++j) acc2[j][ntl] = mfma(wb[j][ks], b, acc2[j][ntl]);
            }
        }
#pragma unroll
        for (int ks = 0; ks < KSe; ++ks) wa[ks] = wa_n[ks];
#pragma unroll
        for (int j = 0; j < MPW; ++j)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) wb[j][ks] = wb_n[j][ks];
    }

    // h_out = h + Wc v + bc
    uint2* hout = reinterpret_cast<uint2*>(a.h_out) + (size_t)img * a.Hf * a.Wf * c4n;
#pragma unroll
    for (int j = 0; j < MPW; ++j) {
        const int t = w + 4 * j;
        if (t >= MTc) break;
        const int o = t * 16 + 4 * g;
        const float bc0 = a.bc[o], bc1 = a.bc[o + 1], bc2 = a.bc[o + 2], bc3 = a.bc[o + 3];
#pragma unroll
        for (int ntl = 0; ntl < 2; ++ntl) {
            const int px = (2 * half + ntl) * 16 + n, ty = px >> 3, tx = px & 7, gy = y0 + ty, gx = x0 + tx;
            if (gy >= a.Hf || gx >= a.Wf) continue;
            const float4 sk = unpack4(*reinterpret_cast<const uint2*>(hl + ((ty + 1) * kIrHW + tx + 1) * ldh + o));
            hout[((size_t)gy * a.Wf + gx) * c4n + (o >> 2)] =
                pack4(acc2[j][ntl][0] + bc0 + sk.x, acc2[j][ntl][1] + bc1 + sk.y, acc2[j][ntl][2] + bc2 + sk.z,
                      acc2[j][ntl][3] + bc3 + sk.w);
        }
    }
}

// ---------------------------------------------------------- fused encoder --

// One workgroup per 8 x 8 tile of encoder outputs.  Working backwards from the
// tile: the second depthwise layer (stride 2) needs e2 on 17 x 17 positions,
// which the first 1x1 makes pointwise from e1 on the same positions, which the
// first depthwise layer (stride 2) makes from the packed planes on 35 x 35
// positions.  Every intermediate stays in LDS (float32 holding the bfloat16
// values the layer-by-layer path stores; zero outside the image, the zero
// padding of the next depthwise layer); the last 1x1 runs on MFMA.
constexpr int kEncT = 8, kEncE2 = 2 * kEncT + 1, kEncA0 = 2 * kEncE2 + 1;
constexpr int kEncThreads = 512;   // eight waves

__global__ __launch_bounds__(kEncThreads) void encoder_kernel(EncArgs a)
{
    extern __shared__ __align__(16) float fl[];
    const int CE = a.ce;
    float* a0 = fl;                                        // [35 * 35][4]
    float* e1 = a0 + kEncA0 * kEncA0 * 4;                  // [17 * 17][4]
    float* e2 = e1 + kEncE2 * kEncE2 * 4;                  // [17 * 17][CE]
    float* wv = e2 + kEncE2 * kEncE2 * CE;                 // w0 [4][9], b0 [4], w1 [CE][4], b1, w2 [CE][9], b2, b3
    float* w0 = wv;
    float* b0 = w0 + 36;
    float* w1 = b0 + 4;
    float* b1 = w1 + CE * 4;
    float* w2 = b1 + CE;
    float* b2 = w2 + CE * 9;
    float* b3 = b2 + CE;
    const int ldc = CE + 8;
    uint16_t* e3 = reinterpret_cast<uint16_t*>(b3 + CE);  // [64][CE + 8] bfloat16 (MFMA B operand rows)

    const int tiles_x = (a.Wf + kEncT - 1) / kEncT, tiles_y = (a.Hf + kEncT - 1) / kEncT;
    const int img = blockIdx.x / (tiles_x * tiles_y), tr = blockIdx.x - img * tiles_x * tiles_y;
    const int Y0 = (tr / tiles_x) * kEncT, X0 = (tr % tiles_x) * kEncT;
    const int tid = threadIdx.x, nt = blockDim.x;

    for (int e = tid; e < 40 + CE * 15 + CE; e += nt) {
        float v;
        if (e < 36) v = a.w0[e];
        else if (e < 40) v = a.b0[e - 36];
        else if (e < 40 + CE * 4) v = bf2f(f2bf(a.w1[e - 40]));           // the 1x1 weights are used as bfloat16
        else if (e < 40 + CE * 5) v = a.b1[e - 40 - CE * 4];
        else if (e < 40 + CE * 14) v = a.w2[e - 40 - CE * 5];
        else if (e < 40 + CE * 15) v = a.b2[e - 40 - CE * 14];
        else v = a.b3[e - 40 - CE * 15];
        wv[e] = v;
    }
    // packed planes (v - 2048) / 1024 on 35 x 35 positions from packed (4 Y0 - 3, 4 X0 - 3);
    // a thread issues all of its mosaic loads before converting and writing LDS
    const uint16_t* m = a.mosaic + img * a.img_stride;
    {
        constexpr int kPl = (kEncA0 * kEncA0 + kEncThreads - 1) / kEncThreads;
        uint16_t qv[kPl][4];
        bool in[kPl];
#pragma unroll
        for (int u = 0; u < kPl; ++u) {
            const int e = tid + kEncThreads * u, r = e / kEncA0, c = e - r * kEncA0;
            const int py = 4 * Y0 - 3 + r, px = 4 * X0 - 3 + c;
            in[u] = e < kEncA0 * kEncA0 && py >= 0 && py < a.Hp && px >= 0 && px < a.Wp;
            qv[u][0] = qv[u][1] = qv[u][2] = qv[u][3] = 0;
            if (in[u]) {
                const uint16_t* q = m + (int64_t)(2 * py) * a.pitch + 2 * px;
                qv[u][0] = q[0];
                qv[u][1] = q[1];
                qv[u][2] = q[a.pitch];
                qv[u][3] = q[a.pitch + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < kPl; ++u) {
            const int e = tid + kEncThreads * u;
            if (e >= kEncA0 * kEncA0) break;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (in[u]) {
                const float k = 1.f / 1024.f;
                v = unpack4(pack4(((float)qv[u][0] - 2048.f) * k, ((float)qv[u][1] - 2048.f) * k,
                                  ((float)qv[u][2] - 2048.f) * k, ((float)qv[u][3] - 2048.f) * k));
            }
            *reinterpret_cast<float4*>(a0 + 4 * e) = v;
        }
    }
    __syncthreads();
    // e1: depthwise stride 2 of the planes on 17 x 17 positions from (2 Y0 - 1, 2 X0 - 1)
    for (int e = tid; e < kEncE2 * kEncE2; e += nt) {
        const int r = e / kEncE2, c = e - r * kEncE2;
        const int gy = 2 * Y0 - 1 + r, gx = 2 * X0 - 1 + c;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gy >= 0 && gy < a.H1 && gx >= 0 && gx < a.W1) {
            float acc[4] = {b0[0], b0[1], b0[2], b0[3]};
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const float4 x = *reinterpret_cast<const float4*>(a0 + 4 * ((2 * r + ky) * kEncA0 + 2 * c + kx));
                    const int t = 3 * ky + kx;
                    acc[0] += w0[t] * x.x;
                    acc[1] += w0[9 + t] * x.y;
                    acc[2] += w0[18 + t] * x.z;
                    acc[3] += w0[27 + t] * x.w;
                }
            v = unpack4(pack4(relu6f(acc[0]), relu6f(acc[1]), relu6f(acc[2]), relu6f(acc[3])));
        }
        *reinterpret_cast<float4*>(e1 + 4 * e) = v;
    }
    __syncthreads();
    // e2: 1x1 4 -> CE on the same positions (zero outside the image)
    for (int e = tid; e < kEncE2 * kEncE2 * CE; e += nt) {
        const int p = e / CE, o = e - p * CE;
        const int r = p / kEncE2, c = p - r * kEncE2;
        const int gy = 2 * Y0 - 1 + r, gx = 2 * X0 - 1 + c;
        float v = 0.f;
        if (gy >= 0 && gy < a.H1 && gx >= 0 && gx < a.W1) {
            const float4 x = *reinterpret_cast<const float4*>(e1 + 4 * p);
            const float* w = w1 + 4 * o;
            v = bf2f(f2bf(relu6f(b1[o] + w[0] * x.x + w[1] * x.y + w[2] * x.z + w[3] * x.w)));
        }
        e2[e] = v;
    }
    __syncthreads();
    // e3: depthwise stride 2 on the 8 x 8 tile, bfloat16 rows for the MFMA
    for (int e = tid; e < kEncT * kEncT * CE; e += nt) {
        const int p = e / CE, o = e - p * CE;
        const int ty = p >> 3, tx = p & 7;
        float acc = b2[o];
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) acc += w2[o * 9 + 3 * ky + kx] * e2[((2 * ty + ky) * kEncE2 + 2 * tx + kx) * CE + o];
        e3[p * ldc + o] = f2bf(relu6f(acc));
    }
    for (int e = tid; e < kEncT * kEncT * 8; e += nt) e3[(e >> 3) * ldc + CE + (e & 7)] = 0;
    __syncthreads();
    // e4: 1x1 CE -> CE on MFMA; wave w takes pixels 16 (w % 4) .. + 15 and the
    // 16-channel output row tiles w / 4, w / 4 + 2, ...
    const int lane = tid & 63, w = tid >> 6, g = lane >> 4, n = lane & 15;
    const int KS = (CE + 15) >> 4, MT = (CE + 15) >> 4;
    const uint2* wp = reinterpret_cast<const uint2*>(a.w3p);
    const int pg = w & 3, nw = (nt >> 6) >> 2;             // pixel group, waves per pixel group
    const uint16_t* brow = e3 + (16 * pg + n) * ldc + 4 * g;
    const int px = 16 * pg + n, Y = Y0 + (px >> 3), X = X0 + (px & 7);
    const bool inside = Y < a.Hf && X < a.Wf;
    uint2* out = reinterpret_cast<uint2*>(a.out) + ((size_t)img * a.Hf * a.Wf + (size_t)Y * a.Wf + X) * (CE >> 2);
    for (int t = w >> 2; t < MT; t += nw) {
        v4f32 acc = (v4f32){0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < KS; ++ks)
            acc = mfma(as_v4(wp[((size_t)t * KS + ks) * 64 + lane]), as_v4(*reinterpret_cast<const uint2*>(brow + 16 * ks)),
                       acc);
        const int o = 16 * t + 4 * g;
        if (inside && o < CE)
            out[o >> 2] = pack4(relu6f(acc[0] + b3[o]), relu6f(acc[1] + b3[o + 1]), relu6f(acc[2] + b3[o + 2]),
                                relu6f(acc[3] + b3[o + 3]));
    }
}

// -------------------------------------------------------------- layout --

// [n][C][HW] (float32 or bfloat16) -> [n][HW][C] bfloat16, through a 64 x 64 LDS
// tile: reads run along pixels, writes along channels (C a multiple of 4).
__global__ __launch_bounds__(256) void to_nhwc_kernel(const void* __restrict__ src, int f32, int C, int HW,
                                                      uint16_t* __restrict__ dst)
{
    __shared__ uint16_t t[64][66];
    const int p0 = blockIdx.x * 64, c0 = blockIdx.y * 64, img = blockIdx.z;
    const int col = 4 * (threadIdx.x & 15);
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int r = (threadIdx.x >> 4) + 16 * pass, c = c0 + r;
        const size_t base = ((size_t)img * C + c) * HW + p0 + col;
        if (f32 && (HW & 3) == 0 && c < C && p0 + col + 3 < HW) {
            const float4 v = *reinterpret_cast<const float4*>(static_cast<const float*>(src) + base);
            t[r][col] = f2bf(v.x);
            t[r][col + 1] = f2bf(v.y);
            t[r][col + 2] = f2bf(v.z);
            t[r][col + 3] = f2bf(v.w);
            continue;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int px = p0 + col + i;
            float v = 0.f;
            if (c < C && px < HW)
                v = f32 ? static_cast<const float*>(src)[base + i] : bf2f(static_cast<const uint16_t*>(src)[base + i]);
            t[r][col + i] = f2bf(v);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int idx = threadIdx.x + 256 * k, px = idx >> 4, c4 = idx & 15;
        const int c = c0 + 4 * c4;
        if (p0 + px < HW && c < C) {
            uint2 v;
            v.x = (uint32_t)t[4 * c4][px] | (uint32_t)t[4 * c4 + 1][px] << 16;
            v.y = (uint32_t)t[4 * c4 + 2][px] | (uint32_t)t[4 * c4 + 3][px] << 16;
            *reinterpret_cast<uint2*>(dst + ((size_t)img * HW + p0 + px) * C + c) = v;
        }
    }
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

// Blocks of 64 positions x 4 channel quarters (a wave per quarter: 64
// consecutive positions, so every channel row is read 256 bytes at a time).
// Pass 1: per position p, s = sum_c |t| (t = z_target - z_pred, quarters added
// in order); bad = tau >= 0 and s / C > tau (flag stored); counts bad
// positions and takes max |r - t| (order-free, so exact).
__global__ __launch_bounds__(256) void prloss_stats_kernel(const float* __restrict__ r, const float* __restrict__ zp,
                                                           const float* __restrict__ zt, int n, int C, int HW,
                                                           float tau, int32_t* __restrict__ nbad,
                                                           uint32_t* __restrict__ maxbits, uint8_t* __restrict__ flags)
{
    __shared__ float ss[4][64];
    __shared__ float wm[4];
    const int j = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int P = n * HW, p = blockIdx.x * 64 + j;
    float s = 0.f, mx = 0.f;
    if (p < P) {
        const int img = p / HW, hw = p - img * HW;
        const size_t base = (size_t)img * C * HW + hw;
        const int c0 = q * C / 4, c1 = (q + 1) * C / 4;
#pragma unroll 4
        for (int c = c0; c < c1; ++c) {
            const size_t i = base + (size_t)c * HW;
            const float t = zt[i] - zp[i];
            s += fabsf(t);
            mx = fmaxf(mx, fabsf(r[i] - t));
        }
    }
    ss[q][j] = s;
    mx = wave_max(mx);
    if (j == 0) wm[q] = mx;
    __syncthreads();
    int bad = 0;
    if (q == 0 && p < P) {
        bad = tau >= 0.f && (((ss[0][j] + ss[1][j]) + ss[2][j]) + ss[3][j]) / (float)C > tau;
        flags[p] = (uint8_t)bad;
    }
    const int cnt = __syncthreads_count(bad);
    if (threadIdx.x == 0) {
        if (cnt) atomicAdd(nbad, cnt);
        atomicMax(maxbits, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
    }
}

// Pass 2: loss terms and dr = dloss/dr (bfloat16, [n][C][HW]); partial[block] =
// the block's loss, summed in a fixed tree order.
__global__ __launch_bounds__(256) void prloss_grad_kernel(const float* __restrict__ r, const float* __restrict__ zp,
                                                          const float* __restrict__ zt, int n, int C, int HW, float tau,
                                                          const int32_t* __restrict__ nbad,
                                                          const uint32_t* __restrict__ maxbits,
                                                          const uint8_t* __restrict__ flags, uint16_t* __restrict__ dr,
                                                          float* __restrict__ partial)
{
    __shared__ float red[256];
    const int j = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int P = n * HW, p = blockIdx.x * 64 + j;
    const float cth = 0.2f * __uint_as_float(*maxbits);
    const int nb = *nbad, ng = P - nb;
    float lsum = 0.f;
    if (p < P) {
        const int img = p / HW, hw = p - img * HW;
        const size_t base = (size_t)img * C * HW + hw;
        float wpos = 1.f / (float)P;
        if (tau >= 0.f && nb > 0 && ng > 0) wpos = flags[p] ? 0.5f / (float)nb : 0.5f / (float)ng;
        const float wgt = wpos / (float)C;
        const int c0 = q * C / 4, c1 = (q + 1) * C / 4;
#pragma unroll 4
        for (int c = c0; c < c1; ++c) {
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
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
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

size_t pw_lds_bytes(int KS) { return (size_t)kPx * (KS * 16 + 4) * sizeof(uint16_t); }

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
    const int ntiles = div_up(a.P, kPx);
    const dim3 grid(ntiles < 2048 ? ntiles : 2048);
    // eight waves while the tiles fit in about one round of workgroups, four beyond
    if (ntiles <= 1024) {
        const size_t lds = pw_lds_bytes(a.KS) + (pw_chw_fast(a) ? 8 * 16 * pw_scld(2) * sizeof(float) : 0);
        hipError_t e = allow_lds(reinterpret_cast<const void*>(pw_kernel<8>), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pw_kernel<8>, grid, dim3(512), lds, st, a);
    } else {
        const size_t lds = pw_lds_bytes(a.KS) + (pw_chw_fast(a) ? 4 * 16 * pw_scld(4) * sizeof(float) : 0);
        hipError_t e = allow_lds(reinterpret_cast<const void*>(pw_kernel<4>), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pw_kernel<4>, grid, dim3(256), lds, st, a);
    }
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
    const int rows = a.P > 0 ? nwg : 0, mw = a.cout * a.cin;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(div_up(mw, 64)), dim3(256), 0, st, a.partial, rows, (size_t)mw, mw, 0,
                       gw, gb);
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(div_up(a.cout, 64)), dim3(256), 0, st, a.partial + (size_t)rows * mw,
                       rows, (size_t)a.cout, a.cout, 0, gb, gb);
    return hipGetLastError();
}

// Runs of kRun outputs per thread when that still leaves enough threads to fill the chip, else one.
template <int S, bool GRAD>
static void dw_launch(const uint16_t* x, const float* w, const float* b, const uint16_t* mask, uint16_t* y, int n, int H,
                      int W, int C, int Ho, int Wo, int relu6, hipStream_t st)
{
    const size_t m8 = (size_t)n * Ho * div_up(Wo, kRun) * (C >> 2);
    if (m8 >= (size_t)1 << 17) {
        hipLaunchKernelGGL((dw_fwd_kernel<S, GRAD, kRun>), dim3((unsigned)((m8 + 255) / 256)), dim3(256), 0, st, x, w,
                           b, mask, y, n, H, W, C, Ho, Wo, relu6);
    } else {
        const size_t m1 = (size_t)n * Ho * Wo * (C >> 2);
        hipLaunchKernelGGL((dw_fwd_kernel<S, GRAD, 1>), dim3((unsigned)((m1 + 255) / 256)), dim3(256), 0, st, x, w, b,
                           mask, y, n, H, W, C, Ho, Wo, relu6);
    }
}

hipError_t launch_dw_fwd(const uint16_t* x, const float* w, const float* b, uint16_t* y, int n, int H, int W, int C,
                         int S, int relu6, hipStream_t st)
{
    const int Ho = (H - 1) / S + 1, Wo = (W - 1) / S + 1;
    if ((size_t)n * Ho * Wo * C == 0) return hipSuccess;
    if (S == 1) dw_launch<1, false>(x, w, b, nullptr, y, n, H, W, C, Ho, Wo, relu6, st);
    else dw_launch<2, false>(x, w, b, nullptr, y, n, H, W, C, Ho, Wo, relu6, st);
    return hipGetLastError();
}

hipError_t launch_dw_dgrad(const uint16_t* dy, const float* w, const uint16_t* mask, uint16_t* dx, int n, int H, int W,
                           int C, int S, hipStream_t st)
{
    if ((size_t)n * H * W * C == 0) return hipSuccess;
    if (S == 1) {
        dw_launch<1, true>(dy, w, nullptr, mask, dx, n, H, W, C, H, W, 0, st);
        return hipGetLastError();
    }
    const int Ho = (H - 1) / 2 + 1, Wo = (W - 1) / 2 + 1;
    const size_t m = (size_t)n * H * W * (C >> 2);
    hipLaunchKernelGGL(dw_dgrad2_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, dy, w, mask, dx, n, H, W,
                       C, Ho, Wo);
    return hipGetLastError();
}

// Three workgroups per CU (42 KB of LDS each) over 256 CUs.
int dw_wgrad_nwg(int n, int Ho, int Wo)
{
    const int U = n * Ho * div_up(Wo, kRun);
    return U < 768 ? U : 768;
}

hipError_t launch_dw_wgrad(const uint16_t* x, const uint16_t* dy, float* partial, float* gw, float* gb, int n, int H,
                           int W, int C, int S, hipStream_t st)
{
    const int Ho = (H - 1) / S + 1, Wo = (W - 1) / S + 1;
    const int nwg = dw_wgrad_nwg(n, Ho, Wo);
    if (nwg > 0) {
        const int chunk = div_up(n * Ho * div_up(Wo, kRun), nwg);
        if (S == 1)
            hipLaunchKernelGGL(dw_wgrad_kernel<1>, dim3(nwg), dim3(256), 0, st, x, dy, partial, n, H, W, C, Ho, Wo,
                               chunk);
        else
            hipLaunchKernelGGL(dw_wgrad_kernel<2>, dim3(nwg), dim3(256), 0, st, x, dy, partial, n, H, W, C, Ho, Wo,
                               chunk);
    }
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(div_up(C * 10, 64)), dim3(256), 0, st, partial, nwg, (size_t)C * 10,
                       C * 10, 1, gw, gb);
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

size_t ir_lds_bytes(int ch, int x)
{
    return (size_t)(kIrRows * (ch + kIrPadH) + kIrRows * kIrLd + kIrT * kIrT * kIrLd) * sizeof(uint16_t) +
           (size_t)x * 11 * sizeof(float);
}

bool ir_fused_ok(int ch, int x)
{
    return (ch == 16 || ch == 32 || ch == 48 || ch == 64 || ch == 96 || ch == 128) && x % kIrChunk == 0 &&
           ir_lds_bytes(ch, x) <= 64 * 1024;
}

hipError_t launch_ir_block(const IrArgs& a, hipStream_t st)
{
    const int tiles = a.n * div_up(a.Hf, kIrT) * div_up(a.Wf, kIrT);
    if (tiles == 0) return hipSuccess;
    if (!ir_fused_ok(a.ch, a.x)) return hipErrorInvalidValue;
    const size_t lds = ir_lds_bytes(a.ch, a.x);
    switch (a.ch) {
    case 16: hipLaunchKernelGGL(ir_block_kernel<16>, dim3(tiles), dim3(kIrThreads), lds, st, a); break;
    case 32: hipLaunchKernelGGL(ir_block_kernel<32>, dim3(tiles), dim3(kIrThreads), lds, st, a); break;
    case 48: hipLaunchKernelGGL(ir_block_kernel<48>, dim3(tiles), dim3(kIrThreads), lds, st, a); break;
    case 64: hipLaunchKernelGGL(ir_block_kernel<64>, dim3(tiles), dim3(kIrThreads), lds, st, a); break;
    case 96: hipLaunchKernelGGL(ir_block_kernel<96>, dim3(tiles), dim3(kIrThreads), lds, st, a); break;
    case 128: hipLaunchKernelGGL(ir_block_kernel<128>, dim3(tiles), dim3(kIrThreads), lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static size_t enc_lds_bytes(int ce)
{
    return (size_t)(kEncA0 * kEncA0 * 4 + kEncE2 * kEncE2 * 4 + kEncE2 * kEncE2 * ce + 40 + ce * 16) * sizeof(float) +
           (size_t)kEncT * kEncT * (ce + 8) * sizeof(uint16_t);
}

bool enc_fused_ok(int ce) { return ce % 16 == 0 && ce <= 128 && enc_lds_bytes(ce) <= 158 * 1024; }

hipError_t launch_encoder(const EncArgs& a, hipStream_t st)
{
    if (!enc_fused_ok(a.ce)) return hipErrorInvalidValue;
    const int tiles = a.n * div_up(a.Hf, kEncT) * div_up(a.Wf, kEncT);
    if (tiles == 0) return hipSuccess;
    const size_t lds = enc_lds_bytes(a.ce);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(encoder_kernel), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(encoder_kernel, dim3(tiles), dim3(kEncThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_to_nhwc(const void* src, int f32, int n, int C, int HW, uint16_t* dst, hipStream_t st)
{
    if ((size_t)n * C * HW == 0) return hipSuccess;
    hipLaunchKernelGGL(to_nhwc_kernel, dim3(div_up(HW, 64), div_up(C, 64), n), dim3(256), 0, st, src, f32, C, HW, dst);
    return hipGetLastError();
}

int prloss_blocks(int P) { return div_up(P, 64); }

hipError_t launch_prloss(const float* r, const float* zp, const float* zt, int n, int C, int HW, float tau,
                         int32_t* nbad, uint32_t* maxbits, uint8_t* flags, uint16_t* dr, float* partial, float* loss,
                         hipStream_t st)
{
    const int P = n * HW, nb = prloss_blocks(P);
    hipError_t e = launch_fill_i32(nbad, 1, 0, st);
    if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t*>(maxbits), 1, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prloss_stats_kernel, dim3(nb), dim3(256), 0, st, r, zp, zt, n, C, HW, tau, nbad, maxbits,
                       flags);
    hipLaunchKernelGGL(prloss_grad_kernel, dim3(nb), dim3(256), 0, st, r, zp, zt, n, C, HW, tau, nbad, maxbits, flags,
                       dr, partial);
    hipLaunchKernelGGL(prloss_sum_kernel, dim3(1), dim3(256), 0, st, partial, nb, loss);
    return hipGetLastError();
}

}  // namespace me
