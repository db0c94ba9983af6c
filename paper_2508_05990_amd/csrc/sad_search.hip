// Block-matching stage search with the SAD criterion on gfx950
// (paper Sec. 3.2: SAD matching criterion, one thread group per block of the
// current frame; Sec. 2.2: full search as the predictor-0 special case).
//
// A workgroup owns nb horizontally adjacent blocks of the current frame, four
// waves per block.  The union of their candidate windows in the reference
// frame is staged in LDS (in dy bands when it does not fit), straight from
// global memory to LDS.  The current block's rows are wave-uniform and reach
// SGPRs through scalar loads.  Each lane owns a KY x KX tile of candidates
// (KX horizontally adjacent), so one LDS segment of CW + KX - 1 words feeds
// CW * KX packed v_sad_u16 operations, each of which adds |a-b| for the two
// 16-bit samples of a word (one packed pixel column of one mosaic row).  The
// winner is the minimum of a 64-bit key (SAD, dx^2+dy^2, dy, dx) -- a total
// order, so the argmin is unique and independent of the reduction order: per
// lane, then a wave butterfly, then across the block's waves through LDS.
//
// Blocks of full width take the register-tiled kernel; blocks cut by the
// right frame edge (width < B) take a plain one-candidate-per-lane kernel.
#include "bf16.h"
#include "internal.h"
#include "warp_cell.h"

namespace me {
namespace {

constexpr int kMaxWaves = 16;
// Workgroup size limit the tiled kernel is compiled for (__launch_bounds__):
// at most two blocks (8 waves) per workgroup.
constexpr int kTiledMaxThreads = 512;
constexpr int kWavesPerBlock = 4;         // default waves per block (a launch may use 2 or 8)
constexpr int kMaxPitch = 256;            // words per LDS row (four 64-word chunks)

// The current frame is read-only for the whole launch and every read of it is
// wave-uniform: reading it through the constant address space lets the
// compiler use scalar loads into SGPRs (v_sad_u16 takes one SGPR operand).
typedef const __attribute__((address_space(4))) uint32_t* cptr_t;

__device__ __forceinline__ cptr_t as_const(const uint32_t* p) { return (cptr_t)(p); }

// Workgroups are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous range of work so that neighbouring blocks, which read
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

// Geometry and candidate rectangle of one block.
struct BlockGeo {
    int blk, y0, x0, h, w;
    int dxlo, dxhi, dylo, dyhi;
};

__device__ __forceinline__ void block_geo(const SearchArgs& a, int B, int blk, BlockGeo& g)
{
    const int bi = blk / a.bw, bj = blk - bi * a.bw;
    g.blk = blk;
    g.y0 = bi * B;
    g.x0 = bj * B;
    g.h = min(B, a.Hp - g.y0);
    g.w = min(B, a.Wp - g.x0);
    int px = 0, py = 0;
    if (a.pred) {
        const int pb = a.pred_ratio > 1 ? (bi / a.pred_ratio) * a.pred_bw + bj / a.pred_ratio : blk;
        px = a.pred[2 * pb];
        py = a.pred[2 * pb + 1];
    } else if (a.net) {                         // clamp(rint(8 o), -limit, limit), ties to even
        const float lim = (float)a.limit;
        const int nblk = a.bh * a.bw;
        px = (int)fminf(fmaxf(rintf(8.0f * a.net[blk]), -lim), lim);
        py = (int)fminf(fmaxf(rintf(8.0f * a.net[nblk + blk]), -lim), lim);
    }
    // radius around the predictor, the +-limit box, displaced block in frame
    g.dxlo = max(max(px - a.R, -a.limit), -g.x0);
    g.dxhi = min(min(px + a.R, a.limit), a.Wp - g.x0 - g.w);
    g.dylo = max(max(py - a.R, -a.limit), -g.y0);
    g.dyhi = min(min(py + a.R, a.limit), a.Hp - g.y0 - g.h);
}

// Stage reference rows [grow0, grow0 + wrows) x words [gcol0, gcol0 + pitch)
// into LDS, 64 words per wave instruction straight from global memory to LDS
// (no register round trip, no wait per row).  Row addresses are wave-uniform;
// the per-lane column offsets are the same for every row.  Positions outside
// the frame load a clamped in-frame word: such words only ever meet
// candidates that are discarded.  The caller waits (vmcnt) and barriers.
__device__ __forceinline__ void stage_window(const SearchArgs& a, uint32_t* lds, int64_t grow0, int gcol0,
                                             int wrows, int wave, int nw, int lane)
{
    const int pitch = a.lds_pitch;
    const int64_t rmax = 2LL * a.Hp - 1;
    const int cmax = a.Wp - 1;
    int gc[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) gc[ch] = min(gcol0 + ch * 64 + lane, cmax);
    for (int rr = wave; rr < wrows; rr += nw) {
        const int64_t gr = min(grow0 + rr, rmax);
        const uint32_t* src = a.ref + gr * a.ref_pitch;
        uint32_t* dst = lds + rr * pitch;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            if (ch * 64 < pitch && ch * 64 + lane < pitch)
                __builtin_amdgcn_global_load_lds(src + gc[ch], dst + ch * 64, 4, 0, 0);
        }
    }
}

// Rows [grow0, grow0 + nrows) x words [gcol0, gcol0 + width) of src (rows
// src_pitch words apart) into LDS as contiguous rows of `width` words: 64
// words per wave instruction whatever the row width (a narrow window takes a
// few instructions instead of one per row).  Rows past rmax and columns past
// cmax read the nearest in-frame word (only discarded candidates meet them).
// The caller waits (vmcnt).
__device__ __forceinline__ void stage_packed(const uint32_t* src, int64_t src_pitch, int64_t grow0, int gcol0, int width,
                                             int nrows, int64_t rmax, int cmax, uint32_t* lds, int lane)
{
    const int total = nrows * width;
    for (int f0 = 0; f0 < total; f0 += 64) {
        const int f = f0 + lane;
        const int r = f / width, c = f - r * width;
        const int64_t gr = min(grow0 + r, rmax);
        const int gc = min(gcol0 + c, cmax);
        if (f < total) __builtin_amdgcn_global_load_lds(src + gr * src_pitch + gc, lds + f0, 4, 0, 0);
    }
}

__device__ __forceinline__ void write_result(const SearchArgs& a, int blk, uint64_t b)
{
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

// SADs of one lane's KY x KX candidate tile over the 2h mosaic rows of a
// full-width block.  curp: first word of the block in the current frame;
// lbase4: LDS position of the tile's first candidate for block row 0; the
// tile's candidate rows are adjacent, so block row r of candidate row j reads
// LDS row r + 2j.  Walking the block rows of one parity in steps of 2, each
// LDS row is loaded once and kept in a ring of KY segments for the KY
// candidate rows that use it; the next ring slot and the next current-block
// row are requested a step ahead of their use.  The current-block rows
// alternate between two register sets by step parity (the unrolled steps
// come in pairs), so a step's scalar load has the whole step to return and
// no copy between the sets is needed.
template <int CW, int NCH, int KX, int KY>
__device__ __forceinline__ void tile_sads(cptr_t curp, int64_t cur_pitch, int h, const uint4* __restrict__ lbase4,
                                          int pitch4, uint32_t (&acc)[KY][KX])
{
    constexpr int SEGV = (CW + KX - 1 + 3) / 4;
    // Scalar and LDS loads share one wait counter and scalar loads return out
    // of order, so any wait for an LDS read also waits for every scalar load
    // in flight.  With KY >= 3 a step's loads are issued only after its first
    // candidate row's SADs (whose wait then covers just the previous step's
    // loads), and the slot of the tile's last candidate row, filled in the
    // step that uses it, is waited for half a step after its request.  Shorter
    // tiles keep the plain order (loads, then every row): a spare ring slot
    // filled a step ahead cost more in registers than it saved in waits (4x2
    // tiles at 4K R=64 and the batch queue measured slower).
    constexpr bool REORDER = KY >= 3;
    constexpr int RS = KY;                           // ring slots
    constexpr int G = RS % 2 == 0 ? RS : 2 * RS;     // steps per unrolled group: whole ring turns, even
#pragma unroll
    for (int j = 0; j < KY; ++j)
#pragma unroll
        for (int i = 0; i < KX; ++i) acc[j][i] = 0u;

#pragma unroll 1
    for (int q = 0; q < NCH; ++q) {
#pragma unroll 1
        for (int par = 0; par < 2; ++par) {
            const uint4* col4 = lbase4 + par * pitch4 + (q * CW) / 4;   // LDS row par, chunk q
            cptr_t ccol = curp + par * cur_pitch + q * CW;                 // block row par, chunk q
            const int64_t rstep = 2 * cur_pitch;
            uint4 ring[RS][SEGV];                          // slot (r mod RS) holds LDS row 2 r + par
#pragma unroll
            for (int t = 0; t < KY - 1; ++t)
#pragma unroll
                for (int v = 0; v < SEGV; ++v) ring[t][v] = col4[(2 * t) * pitch4 + v];
            uint32_t cA[CW], cB[CW];
#pragma unroll
            for (int k = 0; k < CW; ++k) cA[k] = ccol[k];
            cptr_t nxt = ccol + rstep;                     // block row par + 2 (st + 1)
            // step st (u = st mod G): SADs of candidate rows st .. st + KY - 1 against
            // block row cu; block row par + 2 (st + 1) into cx (the last step rereads
            // row par, which is in the block)
            auto row_sads = [&](const int u, const int j, const uint32_t(&cu)[CW], const int k0, const int k1) {
                uint32_t seg[SEGV * 4];
#pragma unroll
                for (int v = 0; v < SEGV; ++v) {
                    const uint4 t4 = ring[(u + j) % RS][v];
                    seg[4 * v + 0] = t4.x;
                    seg[4 * v + 1] = t4.y;
                    seg[4 * v + 2] = t4.z;
                    seg[4 * v + 3] = t4.w;
                }
#pragma unroll
                for (int k = k0; k < k1; ++k)
#pragma unroll
                    for (int i = 0; i < KX; ++i) acc[j][i] = __builtin_amdgcn_sad_u16(cu[k], seg[k + i], acc[j][i]);
            };
            auto loads = [&](const int u, const int st, uint32_t(&cx)[CW]) {
                if (!REORDER)
#pragma unroll
                    for (int v = 0; v < SEGV; ++v) ring[(u + KY - 1) % RS][v] = col4[(2 * (st + KY - 1)) * pitch4 + v];
                const cptr_t src = st + 1 < h ? nxt : ccol;
#pragma unroll
                for (int k = 0; k < CW; ++k) cx[k] = src[k];
                nxt += rstep;
                if (REORDER)
#pragma unroll
                    for (int v = 0; v < SEGV; ++v) ring[(u + KY - 1) % RS][v] = col4[(2 * (st + KY - 1)) * pitch4 + v];
            };
            auto one = [&](const int u, const int st, const uint32_t(&cu)[CW], uint32_t(&cx)[CW]) {
                if constexpr (!REORDER) {
                    loads(u, st, cx);
#pragma unroll
                    for (int j = 0; j < KY; ++j) row_sads(u, j, cu, 0, CW);
                } else {
                    row_sads(u, 0, cu, 0, CW);
                    __builtin_amdgcn_sched_barrier(0);
                    loads(u, st, cx);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int j = 1; j < KY - 1; ++j) row_sads(u, j, cu, 0, CW);
                    __builtin_amdgcn_sched_barrier(0);
                    row_sads(u, KY - 1, cu, 0, CW);
                }
            };
#pragma unroll 1
            for (int step = 0; step < h; step += G) {
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const int st = step + u;               // block row par + 2 st
                    if (st < h) {
                        if (u & 1) one(u, st, cB, cA);
                        else one(u, st, cA, cB);
                    }
                }
            }
        }
    }
}

// The same tile walk with the current block staged in LDS (rows of B words)
// and read as a broadcast (every lane the same address) into VGPRs: the loop
// then issues only LDS reads, which complete in order, so each wait covers
// exactly the reads it needs (no scalar load in flight behind it).  Per step,
// the ring slot for the tile's last candidate row and the next block row are
// requested first, the candidate rows whose LDS rows are already held are
// summed, and only then does the wave wait for the new slot.
template <int CW, int NCH, int KX, int KY>
__device__ __forceinline__ void tile_sads_cl(const uint4* __restrict__ cur4, int h, const uint4* __restrict__ lbase4,
                                             int pitch4, uint32_t (&acc)[KY][KX])
{
    constexpr int B = CW * NCH;
    constexpr int SEGV = (CW + KX - 1 + 3) / 4;
    constexpr int CV = CW / 4;                       // uint4 per row chunk of the current block
    constexpr int RP = B / 4;                        // uint4 per current-block row
    constexpr int KY2 = KY % 2 == 0 ? KY : 2 * KY;   // steps per unrolled group (even)
#pragma unroll
    for (int j = 0; j < KY; ++j)
#pragma unroll
        for (int i = 0; i < KX; ++i) acc[j][i] = 0u;

#pragma unroll 1
    for (int q = 0; q < NCH; ++q) {
#pragma unroll 1
        for (int par = 0; par < 2; ++par) {
            const uint4* col4 = lbase4 + par * pitch4 + (q * CW) / 4;   // LDS row par, chunk q
            const uint4* crow = cur4 + par * RP + q * CV;                  // block row par, chunk q
            uint4 ring[KY][SEGV];
#pragma unroll
            for (int t = 0; t < KY - 1; ++t)
#pragma unroll
                for (int v = 0; v < SEGV; ++v) ring[t][v] = col4[(2 * t) * pitch4 + v];
            uint4 cA[CV], cB[CV];
#pragma unroll
            for (int v = 0; v < CV; ++v) cA[v] = crow[v];
            // step st (u = st mod KY2): SADs against block row par + 2 st (cu);
            // block row par + 2 (st + 1) into cx (the last step rereads its own row)
            auto one = [&](const int u, const int st, const uint4(&cu)[CV], uint4(&cx)[CV]) {
#pragma unroll
                for (int v = 0; v < SEGV; ++v) ring[(u + KY - 1) % KY][v] = col4[(2 * (st + KY - 1)) * pitch4 + v];
                const int nx = st + 1 < h ? st + 1 : st;
#pragma unroll
                for (int v = 0; v < CV; ++v) cx[v] = crow[(2 * nx) * RP + v];
                uint32_t c[CW];
#pragma unroll
                for (int v = 0; v < CV; ++v) {
                    c[4 * v + 0] = cu[v].x;
                    c[4 * v + 1] = cu[v].y;
                    c[4 * v + 2] = cu[v].z;
                    c[4 * v + 3] = cu[v].w;
                }
#pragma unroll
                for (int j = 0; j < KY; ++j) {
                    uint32_t seg[SEGV * 4];
#pragma unroll
                    for (int v = 0; v < SEGV; ++v) {
                        const uint4 t4 = ring[(u + j) % KY][v];
                        seg[4 * v + 0] = t4.x;
                        seg[4 * v + 1] = t4.y;
                        seg[4 * v + 2] = t4.z;
                        seg[4 * v + 3] = t4.w;
                    }
#pragma unroll
                    for (int k = 0; k < CW; ++k)
#pragma unroll
                        for (int i = 0; i < KX; ++i) acc[j][i] = __builtin_amdgcn_sad_u16(c[k], seg[k + i], acc[j][i]);
                }
            };
            int step = 0;
#pragma unroll 1
            for (; step + KY2 <= h; step += KY2) {
#pragma unroll
                for (int u = 0; u < KY2; ++u) {
                    if (u & 1) one(u, step + u, cB, cA);
                    else one(u, step + u, cA, cB);
                }
            }
#pragma unroll
            for (int u = 0; u < KY2 - 1; ++u) {              // h not a multiple of KY2
                if (step + u < h) {
                    if (u & 1) one(u, step + u, cB, cA);
                    else one(u, step + u, cA, cB);
                }
            }
        }
    }
}

// One candidate per lane with a 16-byte aligned LDS column (b128 reads).
template <int CW, int NCH>
__device__ __forceinline__ uint32_t single_sad_aligned(cptr_t curp, int64_t cur_pitch, int rows2,
                                                       const uint4* __restrict__ lbase4, int pitch4)
{
    uint32_t s = 0u;
    for (int r = 0; r < rows2; ++r) {
        cptr_t crow = curp + r * cur_pitch;
        const uint4* l4 = lbase4 + r * pitch4;
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
#pragma unroll
            for (int v = 0; v < CW / 4; ++v) {
                const uint4 t = l4[q * (CW / 4) + v];
                s = __builtin_amdgcn_sad_u16(crow[q * CW + 4 * v + 0], t.x, s);
                s = __builtin_amdgcn_sad_u16(crow[q * CW + 4 * v + 1], t.y, s);
                s = __builtin_amdgcn_sad_u16(crow[q * CW + 4 * v + 2], t.z, s);
                s = __builtin_amdgcn_sad_u16(crow[q * CW + 4 * v + 3], t.w, s);
            }
        }
    }
    return s;
}

// One candidate per lane at any LDS column (word reads).
template <int CW>
__device__ __forceinline__ uint32_t single_sad_full(cptr_t curp, int64_t cur_pitch, int rows2, int nch,
                                                    const uint32_t* __restrict__ lbase, int pitch)
{
    uint32_t s = 0u;
    for (int r = 0; r < rows2; ++r) {
        cptr_t crow = curp + r * cur_pitch;
        const uint32_t* lrow = lbase + r * pitch;
        for (int q = 0; q < nch; ++q) {
#pragma unroll
            for (int k = 0; k < CW; ++k) s = __builtin_amdgcn_sad_u16(crow[q * CW + k], lrow[q * CW + k], s);
        }
    }
    return s;
}

// One candidate per lane over a block of runtime width w.
__device__ __forceinline__ uint32_t single_sad(cptr_t curp, int64_t cur_pitch, int rows2, int w,
                                               const uint32_t* __restrict__ lbase, int pitch)
{
    uint32_t s = 0u;
    for (int r = 0; r < rows2; ++r) {
        cptr_t crow = curp + r * cur_pitch;
        const uint32_t* lrow = lbase + r * pitch;
        for (int k = 0; k < w; ++k) s = __builtin_amdgcn_sad_u16(crow[k], lrow[k], s);
    }
    return s;
}

// Candidates of one block within one dy band, as wave tasks of 64 lanes:
//   main   KY x KX tiles over the first mx = nx - nx % KX columns and the
//          first my = nyb - nyb % KY rows;
//   rows   KX x 1 tiles over the last nyb % KY rows, all columns (the last
//          tile of a row may stick out and is masked);
//   single one candidate per lane over the last nx % KX columns of the first
//          my rows.
// The block's waves take the tasks round-robin, starting at a wave that
// rotates with the block index so the short extra tasks spread over SIMDs.
// lds: LDS word of the block's candidate (dxlo, band row 0) for block row 0.
template <int CW, int NCH, int KX, int KY, bool CL>
__device__ __forceinline__ void block_band(const SearchArgs& a, const BlockGeo& g, int y0c, int nyb, int wib,
                                           const uint32_t* lds, int pitch, int lane, uint64_t& best,
                                           const uint4* cur4)
{
    const uint4* lds4 = reinterpret_cast<const uint4*>(lds);
    const int pitch4 = pitch >> 2;
    const int nx = g.dxhi - g.dxlo + 1;
    const int txn = nx / KX, mx = txn * KX, rx = nx - mx;
    const int txr = (nx + KX - 1) / KX;
    const int tyn = nyb / KY, myb = tyn * KY, ryb = nyb - myb;
    const int n_main = txn * tyn;
    // remainder rows (below the main tiles): KX x 1 tiles, or with a.rs single
    // candidates after the remainder columns (lanes spread more evenly over
    // the block's waves when a tile row would give one wave a long extra task)
    const int n_rows = a.rs ? 0 : txr * ryb;
    const int n_single = rx * myb;
    const int n_single2 = a.rs ? ryb * nx : 0;
    const int t_main = (n_main + 63) >> 6;
    const int t_rows = t_main + ((n_rows + 63) >> 6);
    const int t_single = t_rows + ((n_single + 63) >> 6);
    const int tasks = t_single + ((n_single2 + 63) >> 6);
    cptr_t curp = as_const(a.cur + 2LL * g.y0 * a.cur_pitch + g.x0);
    const int wpb = a.wpb;
    const int first = (wib + wpb - g.blk % wpb) % wpb;
    for (int task = first; task < tasks; task += wpb) {
        if (task < t_main) {
            const int t = task * 64 + lane;
            const bool active = t < n_main;
            const int tt = active ? t : task * 64;
            const int tyl = tt / txn, tx = tt - tyl * txn;
            uint32_t acc[KY][KX];
            if (CL)
                tile_sads_cl<CW, NCH, KX, KY>(cur4, g.h, lds4 + (2 * tyl * KY) * pitch4 + (tx * KX) / 4, pitch4, acc);
            else
                tile_sads<CW, NCH, KX, KY>(curp, a.cur_pitch, g.h, lds4 + (2 * tyl * KY) * pitch4 + (tx * KX) / 4,
                                           pitch4, acc);
            if (active) {
#pragma unroll
                for (int j = 0; j < KY; ++j)
#pragma unroll
                    for (int i = 0; i < KX; ++i) {
                        const uint64_t key = make_key(acc[j][i], g.dxlo + tx * KX + i, g.dylo + y0c + tyl * KY + j);
                        best = key < best ? key : best;
                    }
            }
        } else if (task < t_rows) {
            const int t = (task - t_main) * 64 + lane;
            const bool active = t < n_rows;
            const int tt = active ? t : (task - t_main) * 64;
            const int ry = tt / txr, tx = tt - ry * txr;
            const int cy = myb + ry;
            uint32_t acc[1][KX];
            if (CL)
                tile_sads_cl<CW, NCH, KX, 1>(cur4, g.h, lds4 + (2 * cy) * pitch4 + (tx * KX) / 4, pitch4, acc);
            else
                tile_sads<CW, NCH, KX, 1>(curp, a.cur_pitch, g.h, lds4 + (2 * cy) * pitch4 + (tx * KX) / 4, pitch4, acc);
            if (active) {
#pragma unroll
                for (int i = 0; i < KX; ++i) {
                    if (tx * KX + i < nx) {
                        const uint64_t key = make_key(acc[0][i], g.dxlo + tx * KX + i, g.dylo + y0c + cy);
                        best = key < best ? key : best;
                    }
                }
            }
        } else if (task >= t_single) {
            const int t = (task - t_single) * 64 + lane;
            const bool active = t < n_single2;
            const int tt = active ? t : (task - t_single) * 64;
            const int cy = myb + tt / nx, cx = tt - (tt / nx) * nx;
            const uint32_t sad = single_sad_full<CW>(curp, a.cur_pitch, 2 * g.h, NCH, lds + 2 * cy * pitch + cx, pitch);
            if (active) {
                const uint64_t key = make_key(sad, g.dxlo + cx, g.dylo + y0c + cy);
                best = key < best ? key : best;
            }
        } else {
            const int t = (task - t_rows) * 64 + lane;
            const bool active = t < n_single;
            const int tt = active ? t : (task - t_rows) * 64;
            const int cy = tt / rx, cx = mx + (tt - cy * rx);
            uint32_t sad;
            if (rx == 1)                               // the column is 16-byte aligned (mx % 4 == 0)
                sad = single_sad_aligned<CW, NCH>(curp, a.cur_pitch, 2 * g.h, lds4 + (2 * cy) * pitch4 + cx / 4,
                                                  pitch4);
            else
                sad = single_sad_full<CW>(curp, a.cur_pitch, 2 * g.h, NCH, lds + 2 * cy * pitch + cx, pitch);
            if (active) {
                const uint64_t key = make_key(sad, g.dxlo + cx, g.dylo + y0c + cy);
                best = key < best ? key : best;
            }
        }
    }
}

// Tiled search of the full-width blocks [first_blk, first_blk + nblk) of one
// block row by the whole workgroup (4 waves per block; all threads call it).
// Fused warp: the cells of block blk of wout = Warp(wz, MV) for the block's
// final key (the vector write_result stores), threads t = 0..nt-1 of the
// block.  A thread keeps one cell (taps and weights computed once) and walks
// channels t / ncell, + nt / ncell, ..., loading four channels' taps before
// using them, as the warp kernel does; same arithmetic, so the same bits.
template <bool BF16>
__device__ void warp_block_t(const SearchArgs& a, int blk, uint64_t best, int t, int nt)
{
    const int dx = best == ~0ull ? 0 : (int)(best & 0xffu) - 128;
    const int dy = best == ~0ull ? 0 : (int)((best >> 8) & 0xffu) - 128;
    const int cells = a.block / a.ws;
    const int bi = blk / a.bw, bj = blk - bi * a.bw;
    const int i0 = bi * cells, j0 = bj * cells;
    const int nci = min(cells, a.wHf - i0), ncj = min(cells, a.wWf - j0);
    if (nci <= 0 || ncj <= 0) return;
    const int ncell = nci * ncj;
    const int lanes_per_ch = nt / ncell;                  // threads sharing a cell, on different channels
    if (lanes_per_ch == 0) {
        // more cells than threads (a block of 64 with cells of 1 or 2): one item at a time
        const size_t plane = (size_t)a.wHf * a.wWf;
        for (int item = t; item < a.wC * ncell; item += nt) {
            const int c = item / ncell, k = item - c * ncell;
            const int i = i0 + k / ncj, j = j0 + k % ncj;
            const WarpTaps tp = warp_taps(i, j, dx, dy, a.ws, a.winv_s, a.wHf, a.wWf);
            const size_t base = (size_t)c * plane, o = base + (size_t)i * a.wWf + j;
            if (BF16) {
                const uint16_t* p = static_cast<const uint16_t*>(a.wz) + base;
                static_cast<uint16_t*>(a.wout)[o] =
                    f2bf(warp_mix(tp, bf2f(p[tp.o00]), bf2f(p[tp.o01]), bf2f(p[tp.o10]), bf2f(p[tp.o11])));
            } else {
                const float* p = static_cast<const float*>(a.wz) + base;
                static_cast<float*>(a.wout)[o] = warp_mix(tp, p[tp.o00], p[tp.o01], p[tp.o10], p[tp.o11]);
            }
        }
        return;
    }
    const int k = t % ncell, c0 = t / ncell;
    if (c0 >= lanes_per_ch) return;
    const int i = i0 + k / ncj, j = j0 + k % ncj;
    const WarpTaps tp = warp_taps(i, j, dx, dy, a.ws, a.winv_s, a.wHf, a.wWf);
    const size_t plane = (size_t)a.wHf * a.wWf, cell = (size_t)i * a.wWf + j;
    for (int cb = c0; cb < a.wC; cb += 4 * lanes_per_ch) {
        float v[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int c = cb + u * lanes_per_ch;
            c = c < a.wC ? c : a.wC - 1;
            const size_t base = (size_t)c * plane;
            if (BF16) {
                const uint16_t* p = static_cast<const uint16_t*>(a.wz) + base;
                v[u][0] = bf2f(p[tp.o00]);
                v[u][1] = bf2f(p[tp.o01]);
                v[u][2] = bf2f(p[tp.o10]);
                v[u][3] = bf2f(p[tp.o11]);
            } else {
                const float* p = static_cast<const float*>(a.wz) + base;
                v[u][0] = p[tp.o00];
                v[u][1] = p[tp.o01];
                v[u][2] = p[tp.o10];
                v[u][3] = p[tp.o11];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = cb + u * lanes_per_ch;
            if (c >= a.wC) break;
            const float r = warp_mix(tp, v[u][0], v[u][1], v[u][2], v[u][3]);
            const size_t o = (size_t)c * plane + cell;
            if (BF16) static_cast<uint16_t*>(a.wout)[o] = f2bf(r);
            else static_cast<float*>(a.wout)[o] = r;
        }
    }
}

__device__ __forceinline__ void warp_block(const SearchArgs& a, int blk, uint64_t best, int t, int nt)
{
    if (a.wbf16) warp_block_t<true>(a, blk, best, t, nt);
    else warp_block_t<false>(a, blk, best, t, nt);
}

// Stage the current frame's rows [2 y0, 2 y0 + 2h) x words [x0, x0 + B) of
// the group's blocks into LDS at `dst` (block m at m * 2B * B words, rows of B
// words), 64 consecutive LDS words per wave instruction; rows past 2h load
// row 2h - 1 (never read).  The caller waits (vmcnt) and barriers.
template <int B>
__device__ __forceinline__ void stage_cur(const SearchArgs& a, uint32_t* dst, int y0, int x0, int h, int nblk, int wave,
                                          int nw, int lane)
{
    constexpr int RPI = 64 / B;                      // rows per 64-word instruction
    constexpr int CHUNKS = B > 64 ? B / 64 : 1;
    constexpr int W = B < 64 ? B : 64;
    const int rows = 2 * B;
    const int per_blk = (rows / (B < 64 ? RPI : 1)) * CHUNKS;
    for (int it = wave; it < nblk * per_blk; it += nw) {
        const int m = it / per_blk, k = it - m * per_blk;
        int r, c;
        if (B < 64) {
            r = k * RPI + lane / W;
            c = lane % W;
        } else {
            r = k / CHUNKS;
            c = (k % CHUNKS) * 64 + lane;
        }
        const int rr = min(r, 2 * h - 1);
        const uint32_t* src = a.cur + (2LL * y0 + rr) * a.cur_pitch + x0 + m * B + c;
        __builtin_amdgcn_global_load_lds(src, dst + m * rows * B + (B < 64 ? k * 64 : r * B + (k % CHUNKS) * 64),
                                         4, 0, 0);
    }
}

template <int CW, int NCH, int KX, int KY, bool CL>
__device__ __forceinline__ void run_tiled(const SearchArgs& a, int first_blk, int nblk, uint32_t* lds, uint64_t* red)
{
    constexpr int B = CW * NCH;
    const int tid = threadIdx.x;
    const int nw = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int pitch = a.lds_pitch;
    BlockGeo g0;
    block_geo(a, B, first_blk, g0);
    const int wpb = a.wpb;                          // waves per block
    const int mine = wave / wpb;                    // this wave's block within the group
    const int wib = wave - mine * wpb;
    const bool has_block = mine < nblk;
    BlockGeo g;
    block_geo(a, B, first_blk + (has_block ? mine : 0), g);
    const int left = g0.x0 + g0.dxlo;               // frame column of LDS column 0

    uint64_t best = ~0ull;
    // the blocks of a group share y0, h and (without predictors) the dy range
    if (g0.dylo <= g0.dyhi && g0.dxlo <= g0.dxhi) {
        const int ny = g0.dyhi - g0.dylo + 1;
        const int band = a.band_ty * KY;            // candidate rows per band (multiple of KY)
        for (int y0c = 0; y0c < ny; y0c += band) {
            const int nyb = min(band, ny - y0c);
            __syncthreads();
            stage_window(a, lds, 2LL * (g0.y0 + g0.dylo + y0c), left, 2 * (g0.h + nyb - 1), wave, nw, lane);
            if (CL && y0c == 0) stage_cur<B>(a, lds + a.cur_lds, g0.y0, g0.x0, g0.h, nblk, wave, nw, lane);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (has_block && g.dxlo <= g.dxhi)
                block_band<CW, NCH, KX, KY, CL>(a, g, y0c, nyb, wib, lds + (g.x0 + g.dxlo - left), pitch, lane, best,
                                                reinterpret_cast<const uint4*>(lds + a.cur_lds + mine * 2 * B * B));
        }
    }
    best = wave_min_u64(best);
    if (lane == 0) red[wave] = best;
    __syncthreads();
    if (has_block && wib == 0 && lane == 0) {
        uint64_t b = red[wave];
        for (int k = 1; k < wpb; ++k) b = red[wave + k] < b ? red[wave + k] : b;
        write_result(a, g.blk, b);
    }
    if (a.wz && has_block) {
        const int w0 = mine * wpb;
        uint64_t b = red[w0];
        for (int k = 1; k < wpb; ++k) b = red[w0 + k] < b ? red[w0 + k] : b;
        warp_block(a, g.blk, b, wib * 64 + lane, wpb * 64);
    }
}

// One block of any width, one candidate per lane (a.band_ty candidate rows
// per band, a.lds_pitch words per LDS row); all threads call it.
__device__ __forceinline__ void run_generic(const SearchArgs& a, int blk, uint32_t* lds, uint64_t* red)
{
    BlockGeo g;
    block_geo(a, a.block, blk, g);
    const int tid = threadIdx.x;
    const int nt = blockDim.x, nw = nt >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    uint64_t best = ~0ull;
    if (g.dxlo <= g.dxhi && g.dylo <= g.dyhi) {
        const int nx = g.dxhi - g.dxlo + 1, ny = g.dyhi - g.dylo + 1;
        cptr_t curp = as_const(a.cur + 2LL * g.y0 * a.cur_pitch + g.x0);
        for (int y0c = 0; y0c < ny; y0c += a.band_ty) {
            const int nyb = min(a.band_ty, ny - y0c);
            __syncthreads();
            stage_window(a, lds, 2LL * (g.y0 + g.dylo + y0c), g.x0 + g.dxlo, 2 * (g.h + nyb - 1), wave, nw, lane);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            for (int cand = tid; cand < nx * nyb; cand += nt) {
                const int cy = cand / nx, cx = cand - cy * nx;
                const uint32_t s =
                    single_sad(curp, a.cur_pitch, 2 * g.h, g.w, lds + 2 * cy * a.lds_pitch + cx, a.lds_pitch);
                const uint64_t key = make_key(s, g.dxlo + cx, g.dylo + y0c + cy);
                best = key < best ? key : best;
            }
        }
    }
    best = wave_min_u64(best);
    if (lane == 0) red[wave] = best;
    __syncthreads();
    if (tid == 0) {
        uint64_t b = red[0];
        for (int k = 1; k < nw; ++k) b = red[k] < b ? red[k] : b;
        write_result(a, blk, b);
    }
    if (a.wz) {
        uint64_t b = red[0];
        for (int k = 1; k < nw; ++k) b = red[k] < b ? red[k] : b;
        warp_block(a, blk, b, tid, nt);
    }
}

// The pair a workgroup works on: the launch's own (ref, cur, mv, sad), or,
// in a batch launch, those of job `job` of the launch's job table.
__device__ __forceinline__ SearchArgs for_job(const SearchArgs& a, int job)
{
    SearchArgs b = a;
    const JobPtrs p = a.jobs[job];
    b.ref = p.ref;
    b.cur = p.cur;
    b.mv = p.mv;
    b.sad = p.sad;
    return b;
}

// Full-width blocks, nb per workgroup (nb = 1 when a block list or per-block
// predictors are given, since their candidate rows then differ).  BATCH: the
// grid covers a.n_jobs pairs of one shape, job-major (the paper's batch
// dimension of the (Batch, h, w) grid).
template <int CW, int NCH, int KX, int KY, bool BATCH, bool CL>
__global__ __launch_bounds__(kTiledMaxThreads) void sad_search_kernel(SearchArgs a)
{
    extern __shared__ uint4 lds_dyn[];
    __shared__ uint64_t red[kMaxWaves];
    constexpr int B = CW * NCH;
    int first_blk, nblk;
    if (BATCH) {
        const int groups = (a.ncols + a.nb - 1) / a.nb;
        const int per = a.bh * groups;                 // workgroups per pair
        const int g = xcd_remap(blockIdx.x, gridDim.x);
        const int job = g / per, gid = g - job * per;
        const int bi = gid / groups, gj = gid - bi * groups;
        const int c0 = gj * a.nb;
        first_blk = bi * a.bw + a.col0 + c0;
        nblk = min(a.nb, a.ncols - c0);
        if (min(B, a.Wp - (first_blk % a.bw) * B) != B) return;
        const SearchArgs b = for_job(a, job);
        run_tiled<CW, NCH, KX, KY, CL>(b, first_blk, nblk, reinterpret_cast<uint32_t*>(lds_dyn), red);
        return;
    }
    if (a.list) {
        if ((int)blockIdx.x >= *a.list_n) return;     // whole workgroup leaves
        first_blk = a.list[blockIdx.x];
        nblk = 1;
    } else {
        const int groups = (a.ncols + a.nb - 1) / a.nb;
        const int gid = xcd_remap(blockIdx.x, gridDim.x);
        const int bi = gid / groups, gj = gid - bi * groups;
        const int c0 = gj * a.nb;
        first_blk = bi * a.bw + a.col0 + c0;
        nblk = min(a.nb, a.ncols - c0);
    }
    if (min(B, a.Wp - (first_blk % a.bw) * B) != B) return;   // partial-width blocks: generic kernel
    run_tiled<CW, NCH, KX, KY, CL>(a, first_blk, nblk, reinterpret_cast<uint32_t*>(lds_dyn), red);
}

// Persistent search over a queue of items from many frame pairs of one block
// size (the paper's (Batch, h, w) grid with uneven jobs in one launch): each
// workgroup repeatedly takes the next item -- a group of a job's horizontally
// adjacent full-width blocks -- and searches it with the tiled code above,
// until the queue is empty: workgroup b starts with item b, then draws item
// gridDim.x + ticket from a device counter after each item (so the counter is
// not hit by every workgroup at once).  Items are ordered by job (costlier
// jobs first on the host side), so every workgroup stays busy until the last
// items, whatever the mix of frame sizes and radii.  Each workgroup that had an
// item draws exactly one ticket past the end, so the draw that returns item
// gridDim.x + n_items - 1 is the last one: that workgroup sets the counter back
// to zero for the next launch.
template <int CW, int NCH, int KX, int KY, bool CL>
__global__ __launch_bounds__(kTiledMaxThreads) void sad_queue_kernel(QueueArgs q)
{
    extern __shared__ uint4 lds_dyn[];
    __shared__ uint64_t red[kMaxWaves];
    __shared__ int s_item;
    constexpr int B = CW * NCH;
    int item = blockIdx.x;                            // first item: the workgroup's own; then tickets
    for (;;) {
        if (item >= q.n_items) break;
        int lo = 0, hi = q.n_jobs - 1;                // last job whose first item is <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (q.jobs[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const QueueJob& j = q.jobs[lo];
        SearchArgs a{};
        a.ref = j.ref;
        a.cur = j.cur;
        a.ref_pitch = j.ref_pitch;
        a.cur_pitch = j.cur_pitch;
        a.block = B;
        a.Hp = j.Hp;
        a.Wp = j.Wp;
        a.bh = j.bh;
        a.bw = j.bw;
        a.R = j.R;
        a.limit = j.R;
        a.pred_ratio = 1;
        a.pred_bw = j.bw;
        a.step = 1;
        a.mv = j.mv;
        a.sad = j.sad;
        a.band_ty = j.band_ty;
        a.lds_pitch = j.lds_pitch;
        a.nb = j.nb;
        a.wpb = j.wpb;
        a.cur_lds = j.cur_lds;
        a.rs = j.rs;
        a.col0 = 0;
        a.ncols = j.cols;
        const int it = item - j.item0;
        const int bi = it / j.groups, gj = it - bi * j.groups;
        const int c0 = gj * j.nb;
        run_tiled<CW, NCH, KX, KY, CL>(a, bi * j.bw + c0, min(j.nb, j.cols - c0), reinterpret_cast<uint32_t*>(lds_dyn),
                                       red);
        __syncthreads();                              // the item's window, keys and ticket slot are free
        if (threadIdx.x == 0) s_item = (int)gridDim.x + atomicAdd(q.counter, 1);
        __syncthreads();
        item = __builtin_amdgcn_readfirstlane(s_item);
    }
    if (threadIdx.x == 0 && item == (int)gridDim.x + q.n_items - 1) atomicExch(q.counter, 0);
}

// Blocks cut by the right frame edge: one candidate per lane, runtime width.
template <bool BATCH>
__global__ __launch_bounds__(256) void sad_search_generic(SearchArgs a)
{
    extern __shared__ uint4 lds_dyn[];
    __shared__ uint64_t red[kMaxWaves];
    int blk;
    if (BATCH) {
        const int per = a.bh * a.ncols;
        const int lb = xcd_remap(blockIdx.x, gridDim.x);
        const int job = lb / per, l = lb - job * per;
        const int bi = l / a.ncols;
        blk = bi * a.bw + a.col0 + (l - bi * a.ncols);
        if (min(a.block, a.Wp - (blk % a.bw) * a.block) == a.block) return;
        const SearchArgs b = for_job(a, job);
        run_generic(b, blk, reinterpret_cast<uint32_t*>(lds_dyn), red);
        return;
    }
    if (a.list) {
        if ((int)blockIdx.x >= *a.list_n) return;
        blk = a.list[blockIdx.x];
    } else {
        const int lb = xcd_remap(blockIdx.x, gridDim.x);
        const int bi = lb / a.ncols;
        blk = bi * a.bw + a.col0 + (lb - bi * a.ncols);
    }
    if (min(a.block, a.Wp - (blk % a.bw) * a.block) == a.block) return;   // full width: tiled kernel
    run_generic(a, blk, reinterpret_cast<uint32_t*>(lds_dyn), red);
}

// SAD of one candidate over rows [r0, r1) of a block of width W words (W = 0:
// runtime width w), both operands in LDS: cur rows `cp` words apart (the same
// address in every lane, a broadcast), reference rows `rp` words apart.  The
// next row's words are requested before the current row is summed.
template <int W>
__device__ __forceinline__ uint32_t lds_rows_sad(const uint32_t* cl, int cp, const uint32_t* rl, int rp, int r0,
                                                 int r1, int w)
{
    uint32_t s = 0u;
    if (W > 0) {
        if (r0 >= r1) return 0u;
        uint32_t c[W > 0 ? W : 1], l[W > 0 ? W : 1];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            c[k] = cl[r0 * cp + k];
            l[k] = rl[r0 * rp + k];
        }
        for (int r = r0; r < r1; ++r) {
            const int rn = r + 1 < r1 ? r + 1 : r;
            uint32_t cn[W > 0 ? W : 1], ln[W > 0 ? W : 1];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                cn[k] = cl[rn * cp + k];
                ln[k] = rl[rn * rp + k];
            }
#pragma unroll
            for (int k = 0; k < W; ++k) s = __builtin_amdgcn_sad_u16(c[k], l[k], s);
#pragma unroll
            for (int k = 0; k < W; ++k) {
                c[k] = cn[k];
                l[k] = ln[k];
            }
        }
    } else {
        for (int r = r0; r < r1; ++r)
            for (int k = 0; k < w; ++k) s = __builtin_amdgcn_sad_u16(cl[r * cp + k], rl[r * rp + k], s);
    }
    return s;
}

// Stage searches with a small candidate window (radius <= 4, e.g. the refine
// step of the proposal path): one block per two waves, so a 5x5 window keeps
// most lanes busy where a 4x4 tile per lane would keep one.  The block's rows
// are split between the two waves; each wave stages its half's reference
// window and current-block rows in its own LDS slice of a.band_ty words and
// waits only for its own loads.  Lanes are (candidate, row slice) pairs: with
// nc candidates the half's rows are cut into S slices, the largest power of
// two with S * nc <= 64, and the slices' partial SADs are added with a
// butterfly; the two halves' sums (integers, exact in any order) meet in LDS
// and the first wave of the block takes the minimum key.  Two blocks per
// workgroup.  With a.net (the proposal path), the predictor of each block is
// decoded from the network output in place.
constexpr int kSmallMaxCand = 81;              // (2 x 4 + 1)^2
template <int CW, int NCH, bool BATCH>
__global__ __launch_bounds__(256) void sad_small_kernel(SearchArgs a_in)
{
    extern __shared__ uint4 lds_dyn[];
    __shared__ uint32_t halves[2][2][kSmallMaxCand];   // [block slot][half][candidate]
    constexpr int B = CW * NCH;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int bslot = wave >> 1, half = wave & 1;
    int blk = 0;
    bool active = true;
    SearchArgs a = a_in;
    if (BATCH) {
        const int nblk = a.bh * a.bw;
        const int gb = xcd_remap(blockIdx.x, gridDim.x) * 2 + bslot;
        const int job = gb / nblk;
        active = job < a.n_jobs;
        if (active) {
            blk = gb - job * nblk;
            a = for_job(a_in, job);
        }
    } else if (a.list) {
        const int slot = blockIdx.x * 2 + bslot;
        active = slot < *a.list_n;
        if (active) blk = a.list[slot];
    } else {
        blk = xcd_remap(blockIdx.x, gridDim.x) * 2 + bslot;
        active = blk < a.bh * a.bw;
    }
    BlockGeo g;
    int nc = 0, nx = 1;
    if (active) {
        block_geo(a, B, blk, g);
        if (g.dxlo <= g.dxhi && g.dylo <= g.dyhi) {
            nx = g.dxhi - g.dxlo + 1;
            nc = nx * (g.dyhi - g.dylo + 1);
        }
    }
    if (nc > 0) {
        const int ny = nc / nx, rows = 2 * g.h;
        const int rlo = half ? rows / 2 : 0, hr = (half ? rows : rows / 2) - rlo;   // this wave's mosaic rows
        uint32_t* win = reinterpret_cast<uint32_t*>(lds_dyn) + wave * a.band_ty;
        uint32_t* cblk = win + 2 * (B + 2 * a.R) * a.lds_pitch;        // the half's rows of B words
        stage_packed(a.ref, a.ref_pitch, 2LL * (g.y0 + g.dylo) + rlo, g.x0 + g.dxlo, a.lds_pitch, hr + 2 * (ny - 1),
                     2LL * a.Hp - 1, a.Wp - 1, win, lane);
        stage_packed(a.cur, a.cur_pitch, 2LL * g.y0 + rlo, g.x0, B, hr, 2LL * a.Hp - 1, a.Wp - 1, cblk, lane);
        __builtin_amdgcn_s_waitcnt(0);
        int S = 1;
        while (S < 64 && 2 * S * nc <= 64) S *= 2;
        const int stride = 64 / S;
        const int slice = lane / stride, c0 = lane - slice * stride;
        const int r0 = slice * hr / S, r1 = (slice + 1) * hr / S;
        for (int base = 0; base < nc; base += stride) {
            const int cand = base + c0;
            uint32_t part = 0u;
            if (cand < nc) {
                const int cy = cand / nx, cx = cand - cy * nx;
                const uint32_t* rl = win + 2 * cy * a.lds_pitch + cx;
                part = g.w == B ? lds_rows_sad<B>(cblk, B, rl, a.lds_pitch, r0, r1, B)
                                : lds_rows_sad<0>(cblk, B, rl, a.lds_pitch, r0, r1, g.w);
            }
            for (int off = stride; off < 64; off <<= 1) part += __shfl_xor(part, off, 64);
            if (cand < nc && slice == 0) halves[bslot][half][cand] = part;
        }
    }
    __syncthreads();                                     // every wave reaches it: no early return above
    if (!active || half != 0) return;
    uint64_t best = ~0ull;
    for (int cand = lane; cand < nc; cand += 64) {
        const uint32_t sad = halves[bslot][0][cand] + halves[bslot][1][cand];
        const int cy = cand / nx, cx = cand - cy * nx;
        const uint64_t key = make_key(sad, g.dxlo + cx, g.dylo + cy);
        best = key < best ? key : best;
    }
    best = wave_min_u64(best);
    if (lane == 0) write_result(a, blk, best);
}

__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Stage search with step > 1 (the coarse and intermediate stages of the
// pyramid search, Sec. 3.2): candidates p + step * (u, v), |u|, |v| <= R.
// One block per workgroup of four waves.  The candidate rows are taken in
// bands of a.band_ty rows whose reference rows (2 (h + step (rows - 1))
// mosaic rows of a.lds_pitch words) are staged in LDS.  Lanes work word-
// parallel: a candidate takes B lanes (64 / B candidates per wave), lane k
// holding word k of every row of the current block in registers and reading
// word k of the candidate's reference rows -- consecutive words per
// candidate, so the LDS reads of strided candidates do not pile onto a few
// banks -- and a butterfly over the B lanes adds the columns up.
template <int B>
__global__ __launch_bounds__(256) void sad_step_kernel(SearchArgs a)
{
    extern __shared__ uint4 lds_dyn[];
    __shared__ uint64_t red[kMaxWaves];
    constexpr int G = 64 / B;                       // candidates per wave and pass
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int grp = lane / B, k = lane - grp * B;
    int blk;
    if (a.list) {
        if ((int)blockIdx.x >= *a.list_n) return;     // whole workgroup leaves
        blk = a.list[blockIdx.x];
    } else {
        blk = xcd_remap(blockIdx.x, gridDim.x);
    }
    uint32_t* lds = reinterpret_cast<uint32_t*>(lds_dyn);
    const int s = a.step;
    const int bi = blk / a.bw, bj = blk - bi * a.bw;
    const int y0 = bi * B, x0 = bj * B, h = min(B, a.Hp - y0), w = min(B, a.Wp - x0);
    int px = 0, py = 0;
    if (a.pred) {
        const int pb = a.pred_ratio > 1 ? (bi / a.pred_ratio) * a.pred_bw + bj / a.pred_ratio : blk;
        px = a.pred[2 * pb];
        py = a.pred[2 * pb + 1];
    }
    // u, v such that the displaced block is in the frame and |d| <= limit
    const int xlo = max(-a.limit, -x0), xhi = min(a.limit, a.Wp - x0 - w);
    const int ylo = max(-a.limit, -y0), yhi = min(a.limit, a.Hp - y0 - h);
    const int ulo = max(-a.R, -floor_div(px - xlo, s)), uhi = min(a.R, floor_div(xhi - px, s));
    const int vlo = max(-a.R, -floor_div(py - ylo, s)), vhi = min(a.R, floor_div(yhi - py, s));
    uint64_t best = ~0ull;
    if (ulo <= uhi && vlo <= vhi) {
        const int nx = uhi - ulo + 1, ny = vhi - vlo + 1;
        const int pitch = a.lds_pitch;
        const int rows = 2 * h;
        // column k of the current block, all rows (0 past the block's width)
        uint32_t cur[2 * B];
        {
            const uint32_t* cp = a.cur + 2LL * y0 * a.cur_pitch + x0 + min(k, w - 1);
#pragma unroll
            for (int r = 0; r < 2 * B; ++r) cur[r] = (r < rows && k < w) ? cp[(int64_t)r * a.cur_pitch] : 0u;
        }
        const int gcol = x0 + px + s * ulo;
        for (int cy0 = 0; cy0 < ny; cy0 += a.band_ty) {
            const int nyb = min(a.band_ty, ny - cy0);
            __syncthreads();
            stage_window(a, lds, 2LL * (y0 + py + s * (vlo + cy0)), gcol, 2 * (h + s * (nyb - 1)), wave, 4, lane);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            const int nc = nx * nyb;
            for (int base = 0; base < nc; base += 4 * G) {
                const int cand = base + wave * G + grp;
                const int cc = cand < nc ? cand : nc - 1;
                const int cy = cc / nx, cx = cc - cy * nx;
                const uint32_t* lb = lds + 2 * s * cy * pitch + s * cx + k;
                uint32_t sd = 0u;
                if (rows == 2 * B) {                    // full height; columns past w hold 0 in cur
#pragma unroll
                    for (int r = 0; r < 2 * B; ++r) sd = __builtin_amdgcn_sad_u16(cur[r], lb[r * pitch], sd);
                } else {
#pragma unroll
                    for (int r = 0; r < 2 * B; ++r)
                        if (r < rows) sd = __builtin_amdgcn_sad_u16(cur[r], lb[r * pitch], sd);
                }
                if (k >= w) sd = 0u;                    // lanes past the block's width add nothing
#pragma unroll
                for (int off = B / 2; off >= 1; off >>= 1) sd += __shfl_xor(sd, off, 64);
                if (k == 0 && cand < nc) {
                    const uint64_t key = make_key(sd, px + s * (ulo + cx), py + s * (vlo + cy0 + cy));
                    best = key < best ? key : best;
                }
            }
        }
    }
    best = wave_min_u64(best);
    if (lane == 0) red[wave] = best;
    __syncthreads();
    if (tid == 0) {
        uint64_t b = red[0];
        for (int q = 1; q < 4; ++q) b = red[q] < b ? red[q] : b;
        write_result(a, blk, b);
    }
}

using KernelFn = void (*)(SearchArgs);

template <int CW, int NCH, bool BATCH, bool CL>
KernelFn table_get(int kx, int ky)
{
    if (kx == 4 && ky == 1) return sad_search_kernel<CW, NCH, 4, 1, BATCH, CL>;
    if (kx == 4 && ky == 2) return sad_search_kernel<CW, NCH, 4, 2, BATCH, CL>;
    if (kx == 4 && ky == 4) return sad_search_kernel<CW, NCH, 4, 4, BATCH, CL>;
    if (kx == 8 && ky == 1) return sad_search_kernel<CW, NCH, 8, 1, BATCH, CL>;
    if (kx == 8 && ky == 2) return sad_search_kernel<CW, NCH, 8, 2, BATCH, CL>;
    if (kx == 8 && ky == 4) return sad_search_kernel<CW, NCH, 8, 4, BATCH, CL>;
    return nullptr;
}

template <bool BATCH, bool CL>
KernelFn kernel_for_cl(int B, int kx, int ky)
{
    switch (B) {
    case 8: return table_get<8, 1, BATCH, CL>(kx, ky);
    case 16: return table_get<16, 1, BATCH, CL>(kx, ky);
    case 32: return table_get<16, 2, BATCH, CL>(kx, ky);
    case 64: return table_get<16, 4, BATCH, CL>(kx, ky);
    default: return nullptr;
    }
}

template <bool BATCH>
KernelFn kernel_for(int B, int kx, int ky, int cl)
{
    return cl ? kernel_for_cl<BATCH, true>(B, kx, ky) : kernel_for_cl<BATCH, false>(B, kx, ky);
}

constexpr size_t kLdsCap = 53 * 1024;    // preferred: 3 workgroups per CU
constexpr size_t kLdsMid = 80 * 1024;    // 2 workgroups per CU
constexpr size_t kLdsMax = 158 * 1024;   // gfx950 LDS per workgroup (160 KB) less room for static LDS

hipError_t set_lds(const void* k, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Words per LDS row of the tiled kernel for nb blocks and a candidate window
// of up to n x n: block b's window starts at most b*B words in, and needs
// both its single-candidate reads (n + B - 1 words) and its widest tile
// segment read.  An odd number of 16-byte quads per row spreads lanes that
// read one column of rows 2 apart over the LDS banks.
int tiled_pitch(int B, int n, int kx, int nb)
{
    const int CW = B < 16 ? B : 16;
    const int NCH = B / CW;
    const int segv = (CW + kx - 1 + 3) / 4;
    const int txr = (n + kx - 1) / kx;             // tiles per row, including a partial last one
    int pitch = n + B - 1;
    const int read_end = (txr - 1) * kx + (NCH - 1) * CW + 4 * segv;
    if (read_end > pitch) pitch = read_end;
    pitch += (nb - 1) * B;
    pitch = (pitch + 3) & ~3;
    if (((pitch >> 2) & 1) == 0) pitch += 4;
    return pitch;
}

size_t tiled_bytes(int B, int n, int ky, int band_ty, int pitch)
{
    int rows = band_ty * ky;
    if (rows > n) rows = n;
    return (size_t)2 * (B + rows - 1) * pitch * 4;
}

// LDS bytes of the staged current blocks (2B rows of B words per block).
size_t cur_bytes(int B, int nb, int cl) { return cl ? (size_t)nb * 2 * B * B * 4 : 0; }

}  // namespace

bool tiles_supported(int B, int kx, int ky) { return kernel_for<false>(B, kx, ky, 0) != nullptr; }

namespace {

using QueueFn = void (*)(QueueArgs);

template <int CW, int NCH, bool CL>
QueueFn queue_get(int kx, int ky)
{
    if (kx == 4 && ky == 1) return sad_queue_kernel<CW, NCH, 4, 1, CL>;
    if (kx == 4 && ky == 2) return sad_queue_kernel<CW, NCH, 4, 2, CL>;
    if (kx == 4 && ky == 4) return sad_queue_kernel<CW, NCH, 4, 4, CL>;
    if (kx == 8 && ky == 2) return sad_queue_kernel<CW, NCH, 8, 2, CL>;
    if (kx == 8 && ky == 4) return sad_queue_kernel<CW, NCH, 8, 4, CL>;
    return nullptr;
}

template <bool CL>
QueueFn queue_kernel_for_cl(int B, int kx, int ky)
{
    switch (B) {
    case 8: return queue_get<8, 1, CL>(kx, ky);
    case 16: return queue_get<16, 1, CL>(kx, ky);
    case 32: return queue_get<16, 2, CL>(kx, ky);
    case 64: return queue_get<16, 4, CL>(kx, ky);
    default: return nullptr;
    }
}

QueueFn queue_kernel_for(int B, int kx, int ky, int cl)
{
    return cl ? queue_kernel_for_cl<true>(B, kx, ky) : queue_kernel_for_cl<false>(B, kx, ky);
}

}  // namespace

bool queue_supported(int B, int kx, int ky) { return queue_kernel_for(B, kx, ky, 0) != nullptr; }

bool plan_tiles(int B, int R, size_t lds_cap, TileCfg* cfg)
{
    const int n = 2 * R + 1;
    if (cfg->wpb == 0) cfg->wpb = kWavesPerBlock;
    if (cfg->nb < 1 || (cfg->wpb != 2 && cfg->wpb != 4 && cfg->wpb != 8) ||
        cfg->nb * cfg->wpb * 64 > kTiledMaxThreads)
        return false;
    const int pitch = tiled_pitch(B, n, cfg->kx, cfg->nb);
    if (pitch > kMaxPitch) return false;
    if (cfg->cl != 0 && cfg->cl != 1) return false;
    const size_t cb = cur_bytes(B, cfg->nb, cfg->cl);
    int band = (n + cfg->ky - 1) / cfg->ky;
    while (band > 1 && tiled_bytes(B, n, cfg->ky, band, pitch) + cb > lds_cap) --band;
    const size_t bytes = tiled_bytes(B, n, cfg->ky, band, pitch) + cb;
    if (bytes > lds_cap) return false;
    cfg->band_ty = band;
    cfg->lds_pitch = pitch;
    cfg->lds_bytes = bytes;
    return true;
}

TileCfg list_tiles(int B, int R)
{
    // a listed block takes the whole workgroup: eight waves on 4x2 tiles when
    // its main tiles give each of them a task (a short list then still keeps
    // the chip's SIMDs busy), else four
    TileCfg c{};
    c.kx = 4;
    c.ky = 2;
    c.nb = 1;
    c.rs = 1;
    const int n = 2 * R + 1;
    c.wpb = ((n / 4) * (n / 2) + 63) / 64 >= 8 ? 8 : 4;
    if (plan_tiles(B, R, kLdsMid, &c) || plan_tiles(B, R, kLdsMax, &c)) return c;
    c.wpb = 4;
    if (plan_tiles(B, R, kLdsMid, &c) || plan_tiles(B, R, kLdsMax, &c)) return c;
    return default_tiles(B, R);
}

TileCfg default_tiles(int B, int R)
{
    TileCfg c{};
    c.kx = 4;
    c.rs = 1;
    const int n = 2 * R + 1;
    // Two blocks per workgroup share one window when the radius keeps their
    // window starts 16-byte aligned (R % 4 == 0), within 80 KB (two workgroups
    // per CU).  4x4 tiles only where the block is at least 16 wide, its main
    // tiles give every wave of the block a full 64-lane task and the whole
    // window fits one band; otherwise 4x2 tiles (more, shorter tasks, fewer
    // registers; banded windows at radius 64), which were faster on every
    // other measured (block, radius, frame size).
    if (R % 4 == 0) {
        c.nb = 2;
        if (B >= 16 && (n / 4) * (n / 4) >= 64 * kWavesPerBlock) {
            c.ky = 4;
            if (plan_tiles(B, R, kLdsMid, &c) && c.band_ty * c.ky >= n) return c;
        }
        c.ky = 2;
        if (plan_tiles(B, R, kLdsMid, &c)) return c;
    }
    c.ky = (B >= 16 && (n / 4) * (n / 4) >= 64 * kWavesPerBlock) ? 4 : 2;
    c.nb = 1;
    if (plan_tiles(B, R, kLdsCap, &c) || plan_tiles(B, R, kLdsMid, &c) || plan_tiles(B, R, kLdsMax, &c)) return c;
    return c;
}

// LDS slice per wave of the small-radius kernel: the window (rows of B + 2R
// words, rounded to a multiple of 4) and the current block (2B rows of B
// words); used for radius <= 4 while the slice fits in 32 KB.
bool small_plan(int B, int R, int* pitch, int* words)
{
    if (R > 4) return false;
    const int n = 2 * R + 1;
    const int p = ((B + n - 1) + 3) & ~3;
    const int w = 2 * (B + n - 1) * p + 2 * B * B;  // window, then the current block
    if (p > kMaxPitch || (size_t)w * 4 > 32 * 1024) return false;
    *pitch = p;
    *words = w;
    return true;
}

bool small_search(int B, int R)
{
    int p = 0, w = 0;
    return small_plan(B, R, &p, &w);
}

template <bool BATCH>
KernelFn small_kernel_for(int B)
{
    switch (B) {
    case 8: return sad_small_kernel<8, 1, BATCH>;
    case 16: return sad_small_kernel<16, 1, BATCH>;
    case 32: return sad_small_kernel<16, 2, BATCH>;
    case 64: return sad_small_kernel<16, 4, BATCH>;
    default: return nullptr;
    }
}

KernelFn step_kernel_for(int B)
{
    switch (B) {
    case 8: return sad_step_kernel<8>;
    case 16: return sad_step_kernel<16>;
    case 32: return sad_step_kernel<32>;
    case 64: return sad_step_kernel<64>;
    default: return nullptr;
    }
}

// Strided stage search: window rows of B + 2 R step words (a multiple of 4,
// at most kMaxPitch) and the largest band of candidate rows within 64 KB of
// LDS (160 KB if one row needs more).
bool step_plan(int B, int R, int step, int* pitch, int* band, size_t* bytes)
{
    const int p = ((B + 2 * R * step) + 3) & ~3;
    if (p > kMaxPitch) return false;
    const int n = 2 * R + 1;
    for (size_t cap : {kLdsCap + 11 * 1024, kLdsMax}) {
        int nyb = n;
        while (nyb > 1 && (size_t)2 * (B + step * (nyb - 1)) * p * 4 > cap) --nyb;
        const size_t by = (size_t)2 * (B + step * (nyb - 1)) * p * 4;
        if (by <= cap) {
            *pitch = p;
            *band = nyb;
            *bytes = by;
            return true;
        }
    }
    return false;
}

bool step_supported(int B, int R, int step)
{
    int p = 0, nyb = 0;
    size_t by = 0;
    return step_plan(B, R, step, &p, &nyb, &by);
}

hipError_t launch_sad_search(const SearchArgs& a, const TileCfg& cfg_in, int n_wg, hipStream_t stream, int parts)
{
    const bool batch = a.jobs != nullptr;
    const int64_t njobs = batch ? a.n_jobs : 1;
    if (batch && (a.list || a.n_jobs < 1)) return hipErrorInvalidValue;
    if (a.step < 1) return hipErrorInvalidValue;
    if (a.step > 1) {
        if (batch || a.net) return hipErrorInvalidValue;
        int pitch = 0, nyb = 0;
        size_t bytes = 0;
        KernelFn k = step_kernel_for(a.block);
        if (!k || !step_plan(a.block, a.R, a.step, &pitch, &nyb, &bytes)) return hipErrorInvalidValue;
        hipError_t e = set_lds(reinterpret_cast<const void*>(k), bytes);
        if (e != hipSuccess) return e;
        SearchArgs b = a;
        b.lds_pitch = pitch;
        b.band_ty = nyb;
        const int nw = a.list ? n_wg : a.bh * a.bw;
        if (nw <= 0) return hipSuccess;
        hipLaunchKernelGGL(k, dim3(nw), dim3(256), bytes, stream, b);
        return hipGetLastError();
    }
    int spitch = 0, swords = 0;
    if (small_plan(a.block, a.R, &spitch, &swords)) {
        KernelFn sk = batch ? small_kernel_for<true>(a.block) : small_kernel_for<false>(a.block);
        if (!sk) return hipErrorInvalidValue;
        const size_t bytes = (size_t)4 * swords * 4;    // four waves' slices
        hipError_t e = set_lds(reinterpret_cast<const void*>(sk), bytes);
        if (e != hipSuccess) return e;
        SearchArgs b = a;
        b.lds_pitch = spitch;
        b.band_ty = swords;                             // words per wave slice
        const int64_t nblk = a.list ? n_wg : njobs * a.bh * a.bw;
        if (nblk <= 0) return hipSuccess;
        if ((nblk + 1) / 2 > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(sk, dim3((unsigned)((nblk + 1) / 2)), dim3(256), bytes, stream, b);   // two blocks per workgroup
        return hipGetLastError();
    }
    if (a.net) return hipErrorInvalidValue;          // decoded predictors: small-radius kernel only
    TileCfg cfg = cfg_in;
    if ((a.list || a.pred || (a.R % 4) != 0) && cfg.nb != 1) {   // one block per workgroup
        cfg.nb = 1;
        if (!plan_tiles(a.block, a.R, kLdsCap, &cfg) && !plan_tiles(a.block, a.R, kLdsMid, &cfg) &&
            !plan_tiles(a.block, a.R, kLdsMax, &cfg))
            return hipErrorInvalidValue;
    }
    KernelFn k = batch ? kernel_for<true>(a.block, cfg.kx, cfg.ky, cfg.cl)
                       : kernel_for<false>(a.block, cfg.kx, cfg.ky, cfg.cl);
    const int wpb = cfg.wpb ? cfg.wpb : kWavesPerBlock;
    if (!k || cfg.nb < 1 || (wpb != 2 && wpb != 4 && wpb != 8) || cfg.nb * wpb * 64 > kTiledMaxThreads ||
        (cfg.lds_pitch & 3))
        return hipErrorInvalidValue;
    const int n = 2 * a.R + 1;
    // the shape must cover the widest candidate window of this radius
    const size_t wbytes = tiled_bytes(a.block, n, cfg.ky, cfg.band_ty, cfg.lds_pitch);
    if (cfg.band_ty < 1 || cfg.lds_pitch > kMaxPitch || cfg.lds_pitch < tiled_pitch(a.block, n, cfg.kx, cfg.nb) ||
        wbytes + cur_bytes(a.block, cfg.nb, cfg.cl) > cfg.lds_bytes || cfg.lds_bytes > kLdsMax)
        return hipErrorInvalidValue;
    const int full_cols = a.Wp / a.block;           // block columns of full width
    const bool has_partial = full_cols < a.bw;

    // generic kernel: one candidate per lane, LDS rows of w + n - 1 words
    const int gpitch = ((a.block + n - 1) + 3) & ~3;
    int gband = n;
    while (gband > 1 && (size_t)2 * (a.block + gband - 1) * gpitch * 4 > kLdsCap) --gband;
    size_t gbytes = (size_t)2 * (a.block + gband - 1) * gpitch * 4;
    if (gbytes > kLdsCap) {
        gband = n;
        while (gband > 1 && (size_t)2 * (a.block + gband - 1) * gpitch * 4 > kLdsMax) --gband;
        gbytes = (size_t)2 * (a.block + gband - 1) * gpitch * 4;
    }
    if (has_partial && (gbytes > kLdsMax || gpitch > kMaxPitch)) return hipErrorInvalidValue;
    KernelFn gk = batch ? sad_search_generic<true> : sad_search_generic<false>;

    hipError_t e = set_lds(reinterpret_cast<const void*>(k), cfg.lds_bytes);
    if (e != hipSuccess) return e;
    if (has_partial) {
        e = set_lds(reinterpret_cast<const void*>(gk), gbytes);
        if (e != hipSuccess) return e;
    }
    SearchArgs b = a;
    b.band_ty = cfg.band_ty;
    b.lds_pitch = cfg.lds_pitch;
    b.nb = cfg.nb;
    b.wpb = wpb;
    b.rs = cfg.rs;
    b.cur_lds = (int32_t)(wbytes / 4);              // current blocks after the largest band's window
    SearchArgs c = a;
    c.band_ty = gband;
    c.lds_pitch = gpitch;
    c.nb = 1;
    if (a.list) {
        if (n_wg <= 0) return hipSuccess;
        hipLaunchKernelGGL(k, dim3(n_wg), dim3(wpb * 64), cfg.lds_bytes, stream, b);
        if (has_partial) hipLaunchKernelGGL(gk, dim3(n_wg), dim3(256), gbytes, stream, c);
        return hipGetLastError();
    }
    if (full_cols > 0 && (parts & 1)) {
        b.col0 = 0;
        b.ncols = full_cols;
        const int64_t groups = (full_cols + cfg.nb - 1) / cfg.nb;
        const int64_t grid = njobs * a.bh * groups;
        if (grid > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(cfg.nb * wpb * 64), cfg.lds_bytes, stream, b);
    }
    if (has_partial && (parts & 2)) {
        c.col0 = full_cols;
        c.ncols = 1;
        const int64_t grid = njobs * a.bh;
        if (grid > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(gk, dim3((unsigned)grid), dim3(256), gbytes, stream, c);
    }
    return hipGetLastError();
}

bool plan_queue_job(int B, const TileCfg& tile, size_t lds_cap, QueueJob* j, size_t* lds_bytes)
{
    const int n = 2 * j->R + 1;
    const int main_tasks = ((n / tile.kx) * (n / tile.ky) + 63) / 64;
    // (blocks per item, waves per block), eight waves per workgroup: two blocks
    // of four waves when a block's main tiles give each of its four waves a
    // task, four blocks of two waves for small windows, one block of eight
    // waves when blocks cannot share a window (radius % 4 != 0)
    static const int pref[3][2][2] = {{{1, 8}, {0, 0}}, {{2, 4}, {1, 8}}, {{4, 2}, {2, 4}}};
    const int (*opts)[2] = j->R % 4 ? pref[0] : (main_tasks >= 4 ? pref[1] : pref[2]);
    for (int k = 0; k < 2 && opts[k][0] > 0; ++k) {
        TileCfg c = tile;
        c.nb = opts[k][0];
        c.wpb = opts[k][1];
        if (!plan_tiles(B, j->R, lds_cap, &c)) continue;
        j->nb = c.nb;
        j->wpb = c.wpb;
        j->rs = c.rs;
        j->band_ty = c.band_ty;
        j->lds_pitch = c.lds_pitch;
        j->cur_lds = (int32_t)((c.lds_bytes - cur_bytes(B, c.nb, c.cl)) / 4);
        j->cols = j->Wp / B;
        j->groups = (j->cols + c.nb - 1) / c.nb;
        *lds_bytes = c.lds_bytes;
        return true;
    }
    return false;
}

hipError_t launch_sad_queue(const QueueArgs& q, int B, const TileCfg& tile, size_t lds_bytes, hipStream_t stream)
{
    const QueueFn k = queue_kernel_for(B, tile.kx, tile.ky, tile.cl);
    if (!k || lds_bytes > kLdsMax || q.n_jobs < 1 || !q.counter) return hipErrorInvalidValue;
    if (q.n_items <= 0) return hipSuccess;
    hipError_t e = set_lds(reinterpret_cast<const void*>(k), lds_bytes);
    if (e != hipSuccess) return e;
    int occ = 0, dev = 0, ncu = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, kTiledMaxThreads, lds_bytes)) != hipSuccess ||
        (e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    const int64_t slots = (int64_t)(occ > 0 ? occ : 1) * (ncu > 0 ? ncu : 1);
    const int grid = (int)(slots < q.n_items ? slots : q.n_items);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kTiledMaxThreads), lds_bytes, stream, q);
    return hipGetLastError();
}

}  // namespace me
