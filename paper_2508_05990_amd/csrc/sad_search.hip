// Block-matching stage search with the SAD criterion on gfx950
// (paper Sec. 3.2: SAD matching criterion, one thread group per block of the
// current frame; Sec. 2.2: full search as the predictor-0 special case).
//
// One workgroup owns one block of the current frame.  Its candidate window of
// the reference frame is staged in LDS (in dy bands when it does not fit);
// the current block's rows are wave-uniform and go to SGPRs through scalar
// loads; each lane owns a KY x KX tile of candidates (KX horizontally
// adjacent), so one LDS segment of CW + KX - 1 words feeds CW * KX packed
// v_sad_u16 operations, each of which adds |a-b| for the two 16-bit samples
// of a word (one packed pixel column of one mosaic row).  The winner is the
// minimum of a 64-bit key (SAD, dx^2+dy^2, dy, dx) -- a total order, so the
// argmin is unique and independent of the reduction order: per lane, then a
// wave butterfly, then across waves through LDS.
//
// Blocks of full width take the register-tiled kernel; blocks cut by the
// right frame edge (width < B) take a plain one-candidate-per-lane kernel.
#include "internal.h"

namespace me {
namespace {

constexpr int kMaxWaves = 16;

// Workgroups are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous range of blocks so that neighbouring blocks, which read
// overlapping reference windows, share one L2.
__device__ __forceinline__ int xcd_remap(int bid, int n)
{
    const int xcd = bid & 7, k = bid >> 3;
    const int q = n >> 3, rem = n & 7;
    return xcd * q + min(xcd, rem) + k;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t make_key(uint32_t sad, int dx, int dy)
{
    const uint32_t lo = (uint32_t)(dx * dx + dy * dy) << 16 | (uint32_t)(dy + 128) << 8 | (uint32_t)(dx + 128);
    return (uint64_t)sad << 32 | lo;
}

// Block geometry and candidate rectangle of one workgroup.
struct BlockGeo {
    int blk, y0, x0, h, w;
    int dxlo, dxhi, dylo, dyhi;
};

// Resolve which block this workgroup owns; false if it owns none.
__device__ __forceinline__ bool block_of(const SearchArgs& a, int B, BlockGeo& g)
{
    int blk;
    if (a.list) {
        if ((int)blockIdx.x >= *a.list_n) return false;
        blk = a.list[blockIdx.x];
    } else {
        const int lb = xcd_remap(blockIdx.x, gridDim.x);
        const int bi = lb / a.ncols;
        blk = bi * a.bw + a.col0 + (lb - bi * a.ncols);
    }
    const int bi = blk / a.bw, bj = blk - bi * a.bw;
    g.blk = blk;
    g.y0 = bi * B;
    g.x0 = bj * B;
    g.h = min(B, a.Hp - g.y0);
    g.w = min(B, a.Wp - g.x0);
    int px = 0, py = 0;
    if (a.pred) {
        px = a.pred[2 * blk];
        py = a.pred[2 * blk + 1];
    }
    // radius around the predictor, the +-limit box, displaced block in frame
    g.dxlo = max(max(px - a.R, -a.limit), -g.x0);
    g.dxhi = min(min(px + a.R, a.limit), a.Wp - g.x0 - g.w);
    g.dylo = max(max(py - a.R, -a.limit), -g.y0);
    g.dyhi = min(min(py + a.R, a.limit), a.Hp - g.y0 - g.h);
    return true;
}

// Stage reference rows [grow0, grow0 + wrows) x words [gcol0, gcol0 + wcols)
// into LDS, one wave per row; samples outside the frame read as zero (they
// only ever meet candidates that are discarded).
__device__ __forceinline__ void stage_window(const SearchArgs& a, uint32_t* lds, int64_t grow0, int gcol0,
                                             int wrows, int wcols, int wave, int nw, int lane)
{
    const int64_t rows_in = 2LL * a.Hp;
    for (int rr = wave; rr < wrows; rr += nw) {
        const int64_t gr = grow0 + rr;
        const uint32_t* src = a.ref + gr * a.ref_pitch + gcol0;
        uint32_t* dst = lds + rr * a.lds_pitch;
        const bool row_in = gr < rows_in;
        for (int cc = lane; cc < wcols; cc += 64) {
            uint32_t v = 0u;
            if (row_in && gcol0 + cc < a.Wp) v = src[cc];
            dst[cc] = v;
        }
    }
}

// Reduce the per-lane best keys of the workgroup and write the block result.
__device__ __forceinline__ void finish(const SearchArgs& a, uint64_t best, int blk, uint64_t* red)
{
    const int tid = threadIdx.x, nw = blockDim.x >> 6;
    best = wave_min_u64(best);
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
        uint64_t b = red[0];
        for (int k = 1; k < nw; ++k) b = red[k] < b ? red[k] : b;
        if (b == ~0ull) {
            a.mv[2 * blk] = 0;
            a.mv[2 * blk + 1] = 0;
            a.sad[blk] = -1;
        } else {
            a.mv[2 * blk] = (int16_t)((int)(b & 0xffu) - 128);
            a.mv[2 * blk + 1] = (int16_t)((int)((b >> 8) & 0xffu) - 128);
            a.sad[blk] = (int32_t)(b >> 32);
        }
    }
}

// SADs of one lane's KY x KX candidate tile over the 2h mosaic rows of a
// full-width block.  curp: first word of the block in the current frame;
// lbase4: LDS position of the tile's first candidate for block row 0.
template <int CW, int NCH, int KX, int KY>
__device__ __forceinline__ void tile_sads(const uint32_t* __restrict__ curp, int64_t cur_pitch, int rows2,
                                          const uint4* __restrict__ lbase4, int pitch4, uint32_t (&acc)[KY][KX])
{
    constexpr int SEGV = (CW + KX - 1 + 3) / 4;
#pragma unroll
    for (int j = 0; j < KY; ++j)
#pragma unroll
        for (int i = 0; i < KX; ++i) acc[j][i] = 0u;

    for (int r = 0; r < rows2; ++r) {
        const uint32_t* crow = curp + r * cur_pitch;
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            uint32_t c[CW];
#pragma unroll
            for (int k = 0; k < CW; ++k) c[k] = crow[q * CW + k];
#pragma unroll
            for (int j = 0; j < KY; ++j) {
                const uint4* l4 = lbase4 + (r + 2 * j) * pitch4 + (q * CW) / 4;
                uint32_t seg[SEGV * 4];
#pragma unroll
                for (int v = 0; v < SEGV; ++v) {
                    const uint4 t = l4[v];
                    seg[4 * v + 0] = t.x;
                    seg[4 * v + 1] = t.y;
                    seg[4 * v + 2] = t.z;
                    seg[4 * v + 3] = t.w;
                }
#pragma unroll
                for (int k = 0; k < CW; ++k)
#pragma unroll
                    for (int i = 0; i < KX; ++i) acc[j][i] = __builtin_amdgcn_sad_u16(c[k], seg[k + i], acc[j][i]);
            }
        }
    }
}

template <int CW, int NCH, int KX, int KY>
__global__ __launch_bounds__(kMaxWaves * 64) void sad_search_kernel(SearchArgs a)
{
    extern __shared__ uint4 lds4[];
    __shared__ uint64_t red[kMaxWaves];
    constexpr int B = CW * NCH;
    BlockGeo g;
    if (!block_of(a, B, g)) return;
    if (g.w != B) return;                      // partial-width blocks: generic kernel
    uint32_t* lds = reinterpret_cast<uint32_t*>(lds4);
    const int tid = threadIdx.x;
    const int nt = blockDim.x, nw = nt >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int pitch4 = a.lds_pitch >> 2;

    uint64_t best = ~0ull;
    if (g.dxlo <= g.dxhi && g.dylo <= g.dyhi) {
        const int nx = g.dxhi - g.dxlo + 1, ny = g.dyhi - g.dylo + 1;
        const int txn = (nx + KX - 1) / KX, tyn = (ny + KY - 1) / KY;
        const int wcols = B + txn * KX - 1;
        const uint32_t* curp = a.cur + 2LL * g.y0 * a.cur_pitch + g.x0;
        for (int ty0 = 0; ty0 < tyn; ty0 += a.band_ty) {
            const int bty = min(a.band_ty, tyn - ty0);
            __syncthreads();
            stage_window(a, lds, 2LL * (g.y0 + g.dylo + ty0 * KY), g.x0 + g.dxlo, 2 * (g.h + bty * KY - 1), wcols,
                         wave, nw, lane);
            __syncthreads();
            const int ntiles = txn * bty;
            for (int t0 = wave * 64; t0 < ntiles; t0 += nt) {
                const int t = t0 + lane;
                const bool active = t < ntiles;
                const int tt = active ? t : t0;
                const int tyl = tt / txn, tx = tt - tyl * txn;
                const uint4* lbase4 = lds4 + (2 * tyl * KY) * pitch4 + (tx * KX) / 4;
                uint32_t acc[KY][KX];
                tile_sads<CW, NCH, KX, KY>(curp, a.cur_pitch, 2 * g.h, lbase4, pitch4, acc);
                if (active) {
#pragma unroll
                    for (int j = 0; j < KY; ++j)
#pragma unroll
                        for (int i = 0; i < KX; ++i) {
                            const int dx = g.dxlo + tx * KX + i;
                            const int dy = g.dylo + (ty0 + tyl) * KY + j;
                            if (dx <= g.dxhi && dy <= g.dyhi) {
                                const uint64_t key = make_key(acc[j][i], dx, dy);
                                best = key < best ? key : best;
                            }
                        }
                }
            }
        }
    }
    finish(a, best, g.blk, red);
}

// Blocks cut by the right frame edge: one candidate per lane, runtime width.
__global__ __launch_bounds__(256) void sad_search_generic(SearchArgs a)
{
    extern __shared__ uint4 lds4[];
    __shared__ uint64_t red[kMaxWaves];
    BlockGeo g;
    if (!block_of(a, a.block, g)) return;
    if (g.w == a.block) return;                // full-width blocks: tiled kernel
    uint32_t* lds = reinterpret_cast<uint32_t*>(lds4);
    const int tid = threadIdx.x;
    const int nt = blockDim.x, nw = nt >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    uint64_t best = ~0ull;
    if (g.dxlo <= g.dxhi && g.dylo <= g.dyhi) {
        const int nx = g.dxhi - g.dxlo + 1, ny = g.dyhi - g.dylo + 1;
        const int wcols = g.w + nx - 1;
        const uint32_t* curp = a.cur + 2LL * g.y0 * a.cur_pitch + g.x0;
        for (int y0c = 0; y0c < ny; y0c += a.band_ty) {
            const int nyb = min(a.band_ty, ny - y0c);
            __syncthreads();
            stage_window(a, lds, 2LL * (g.y0 + g.dylo + y0c), g.x0 + g.dxlo, 2 * (g.h + nyb - 1), wcols, wave, nw,
                         lane);
            __syncthreads();
            for (int cand = tid; cand < nx * nyb; cand += nt) {
                const int cy = cand / nx, cx = cand - cy * nx;
                uint32_t s = 0u;
                for (int r = 0; r < 2 * g.h; ++r) {
                    const uint32_t* crow = curp + r * a.cur_pitch;
                    const uint32_t* lrow = lds + (r + 2 * cy) * a.lds_pitch + cx;
                    for (int k = 0; k < g.w; ++k) s = __builtin_amdgcn_sad_u16(crow[k], lrow[k], s);
                }
                const uint64_t key = make_key(s, g.dxlo + cx, g.dylo + y0c + cy);
                best = key < best ? key : best;
            }
        }
    }
    finish(a, best, g.blk, red);
}

using KernelFn = void (*)(SearchArgs);

template <int CW, int NCH>
KernelFn table_get(int kx, int ky)
{
    if (kx == 4 && ky == 1) return sad_search_kernel<CW, NCH, 4, 1>;
    if (kx == 4 && ky == 2) return sad_search_kernel<CW, NCH, 4, 2>;
    if (kx == 4 && ky == 4) return sad_search_kernel<CW, NCH, 4, 4>;
    if (kx == 8 && ky == 1) return sad_search_kernel<CW, NCH, 8, 1>;
    if (kx == 8 && ky == 2) return sad_search_kernel<CW, NCH, 8, 2>;
    if (kx == 8 && ky == 4) return sad_search_kernel<CW, NCH, 8, 4>;
    return nullptr;
}

KernelFn kernel_for(int B, int kx, int ky)
{
    switch (B) {
    case 8: return table_get<8, 1>(kx, ky);
    case 16: return table_get<16, 1>(kx, ky);
    case 32: return table_get<16, 2>(kx, ky);
    case 64: return table_get<16, 4>(kx, ky);
    default: return nullptr;
    }
}

constexpr size_t kLdsCap = 64 * 1024;    // preferred window size: leaves room for 2 workgroups per CU
constexpr size_t kLdsMax = 160 * 1024;   // gfx950 LDS per workgroup

hipError_t set_lds(const void* k, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

bool tiles_supported(int B, int kx, int ky) { return kernel_for(B, kx, ky) != nullptr; }

bool plan_tiles(int B, int nx_max, int ny_max, size_t lds_cap, TileCfg* cfg)
{
    const int CW = B < 16 ? B : 16;
    const int NCH = B / CW;
    const int kx = cfg->kx, ky = cfg->ky;
    const int txn = (nx_max + kx - 1) / kx, tyn = (ny_max + ky - 1) / ky;
    const int segv = (CW + kx - 1 + 3) / 4;
    int pitch = B + txn * kx - 1;
    const int read_end = (txn - 1) * kx + (NCH - 1) * CW + 4 * segv;
    if (read_end > pitch) pitch = read_end;
    pitch = (pitch + 3) & ~3;
    if (pitch % 32 == 0) pitch += 4;   // rows of a band start on different banks
    int band = tyn;
    while (band > 1 && (size_t)2 * (B + band * ky - 1) * pitch * 4 > lds_cap) --band;
    const size_t bytes = (size_t)2 * (B + band * ky - 1) * pitch * 4;
    if (bytes > lds_cap) return false;
    cfg->band_ty = band;
    cfg->lds_pitch = pitch;
    cfg->lds_bytes = bytes;
    return true;
}

TileCfg default_tiles(int B, int R)
{
    TileCfg c{};
    c.kx = 8;
    c.ky = 2;
    const int n = 2 * R + 1;
    const int tiles = ((n + c.kx - 1) / c.kx) * ((n + c.ky - 1) / c.ky);
    const int nw = (tiles + 63) / 64;
    c.nw = nw < 1 ? 1 : (nw > 8 ? 8 : nw);
    if (!plan_tiles(B, n, n, kLdsCap, &c)) plan_tiles(B, n, n, kLdsMax, &c);
    return c;
}

hipError_t launch_sad_search(const SearchArgs& a, const TileCfg& cfg, int n_wg, hipStream_t stream)
{
    KernelFn k = kernel_for(a.block, cfg.kx, cfg.ky);
    if (!k || cfg.nw < 1 || cfg.nw > kMaxWaves || (cfg.lds_pitch & 3)) return hipErrorInvalidValue;
    const int n = 2 * a.R + 1;
    {   // the shape must cover the widest candidate window of this radius
        TileCfg need = cfg;
        if (!plan_tiles(a.block, n, n, cfg.lds_bytes, &need) || need.lds_pitch > cfg.lds_pitch ||
            (size_t)2 * (a.block + cfg.band_ty * cfg.ky - 1) * cfg.lds_pitch * 4 > cfg.lds_bytes)
            return hipErrorInvalidValue;
    }
    const int full_cols = a.Wp / a.block;           // block columns of full width
    const bool has_partial = full_cols < a.bw;

    // generic kernel: one candidate per lane, LDS rows of w + n - 1 words
    int gpitch = ((a.block + n - 1) + 3) & ~3;
    if (gpitch % 32 == 0) gpitch += 4;
    int gband = n;
    while (gband > 1 && (size_t)2 * (a.block + gband - 1) * gpitch * 4 > kLdsCap) --gband;
    size_t gbytes = (size_t)2 * (a.block + gband - 1) * gpitch * 4;
    if (gbytes > kLdsCap) {
        gband = n;
        while (gband > 1 && (size_t)2 * (a.block + gband - 1) * gpitch * 4 > kLdsMax) --gband;
        gbytes = (size_t)2 * (a.block + gband - 1) * gpitch * 4;
    }
    if (has_partial && gbytes > kLdsMax) return hipErrorInvalidValue;

    if (cfg.lds_bytes > kLdsMax) return hipErrorInvalidValue;
    hipError_t e = set_lds(reinterpret_cast<const void*>(k), cfg.lds_bytes);
    if (e != hipSuccess) return e;
    if (has_partial) {
        e = set_lds(reinterpret_cast<const void*>(sad_search_generic), gbytes);
        if (e != hipSuccess) return e;
    }
    SearchArgs b = a;
    b.band_ty = cfg.band_ty;
    b.lds_pitch = cfg.lds_pitch;
    if (a.list) {
        if (n_wg <= 0) return hipSuccess;
        hipLaunchKernelGGL(k, dim3(n_wg), dim3(cfg.nw * 64), cfg.lds_bytes, stream, b);
        if (has_partial) {
            SearchArgs c = a;
            c.band_ty = gband;
            c.lds_pitch = gpitch;
            hipLaunchKernelGGL(sad_search_generic, dim3(n_wg), dim3(256), gbytes, stream, c);
        }
        return hipGetLastError();
    }
    if (full_cols > 0) {
        b.col0 = 0;
        b.ncols = full_cols;
        hipLaunchKernelGGL(k, dim3(a.bh * full_cols), dim3(cfg.nw * 64), cfg.lds_bytes, stream, b);
    }
    if (has_partial) {
        SearchArgs c = a;
        c.band_ty = gband;
        c.lds_pitch = gpitch;
        c.col0 = full_cols;
        c.ncols = 1;
        hipLaunchKernelGGL(sad_search_generic, dim3(a.bh), dim3(256), gbytes, stream, c);
    }
    return hipGetLastError();
}

}  // namespace me
