/*
 * CPU oracle for Bayer-domain block-matching motion estimation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the HIP kernels.
 *
 * What it computes (paper, Sec. 2.2 "Definition" and Sec. 3.2 "Matching
 * Criterion"): for every block of the current frame, the candidate offset in
 * the reference frame whose sum of absolute differences (SAD) is lowest; the
 * motion vector is that offset (position in the reference minus position in
 * the current frame).  Full search (Sec. 2.2, "Block Matching-based ME") is the
 * special case predictor = 0, step = 1.
 *
 * Readings the paper leaves open, fixed here:
 *   - the Bayer mosaic (RGGB at the origin) is viewed as four packed colour
 *     planes, P[c][y][x] = M[2y + (c>>1)][2x + (c&1)]; block sizes, radii and
 *     vectors are in packed-plane pixels and the SAD sums all four planes
 *     unweighted;
 *   - blocks tile the packed frame from the origin, the last row/column of
 *     blocks may be partial and is kept;
 *   - a candidate is kept only if the displaced block lies wholly inside the
 *     reference frame (no padding, no clamping of reads) and both components
 *     of the total vector are within +-limit;
 *   - ties on SAD go to the smaller squared length dx*dx+dy*dy, then the
 *     smaller dy, then the smaller dx: the key (SAD, |d|^2, dy, dx) is a total
 *     order, so the answer is unique;
 *   - the search radius R counts candidates per side, (2R+1)^2 per block,
 *     matching the thread count per block the paper gives in its CUDA
 *     settings (Sec. 4.1).
 *
 * Plain loops, 64-bit accumulation, one OpenMP loop over independent blocks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Packed-plane view of an RGGB mosaic (step A1). planes is [4][H/2][W/2]. */
void oracle_pack_planes(const uint16_t* mosaic, int32_t H, int32_t W, int64_t pitch, uint16_t* planes)
{
    const int32_t Hp = H / 2, Wp = W / 2;
    for (int c = 0; c < 4; ++c) {
        const int ry = c >> 1, rx = c & 1;
        for (int32_t y = 0; y < Hp; ++y)
            for (int32_t x = 0; x < Wp; ++x)
                planes[((int64_t)c * Hp + y) * Wp + x] = mosaic[(int64_t)(2 * y + ry) * pitch + (2 * x + rx)];
    }
}

/* SAD between the current block [y0,y1)x[x0,x1) and the reference block
 * displaced by (dx, dy), summed over the four planes. */
static int64_t block_sad(const uint16_t* ref, const uint16_t* cur, int32_t Hp, int32_t Wp,
                         int32_t y0, int32_t y1, int32_t x0, int32_t x1, int32_t dx, int32_t dy)
{
    int64_t s = 0;
    for (int c = 0; c < 4; ++c) {
        const uint16_t* cp = cur + (int64_t)c * Hp * Wp;
        const uint16_t* rp = ref + (int64_t)c * Hp * Wp;
        for (int32_t y = y0; y < y1; ++y)
            for (int32_t x = x0; x < x1; ++x) {
                int32_t a = cp[(int64_t)y * Wp + x];
                int32_t b = rp[(int64_t)(y + dy) * Wp + (x + dx)];
                s += (a > b) ? (a - b) : (b - a);
            }
    }
    return s;
}

/* Key order (SAD, dx^2+dy^2, dy, dx), lexicographic ascending. */
static int key_less(int64_t sa, int32_t dxa, int32_t dya, int64_t sb, int32_t dxb, int32_t dyb)
{
    if (sa != sb) return sa < sb;
    int32_t ma = dxa * dxa + dya * dya, mb = dxb * dxb + dyb * dyb;
    if (ma != mb) return ma < mb;
    if (dya != dyb) return dya < dyb;
    return dxa < dxb;
}

/*
 * One stage of block matching over packed planes (steps A2 + A3).
 *
 * ref, cur : packed planes [4][Hp][Wp]
 * B        : block size (packed pixels); blocks are bh x bw, bh = ceil(Hp/B)
 * R, step  : candidates d = p + step*(u, v), u, v in [-R, R]
 * pred     : per-block predictor p [bh][bw][2] as (dx, dy), or NULL for p = 0
 * limit    : candidates with |dx| > limit or |dy| > limit are dropped
 * blocks   : optional list of n_blocks block indices (row-major); NULL = all
 * mv, sad  : outputs indexed by block [bh][bw][2] / [bh][bw].  A block with no
 *            valid candidate gets sad = -1 and mv = (0, 0).
 * ops_valid: optional; receives the number of |a-b| terms evaluated, i.e.
 *            sum over blocks of (#valid candidates * #samples in the block)
 * ops_enum : optional; the same count over all (2R+1)^2 enumerated candidates
 *            before the validity test
 * Returns 0, or -1 on bad arguments, -2 if a SAD exceeds INT32_MAX.
 */
int32_t oracle_stage_search(const uint16_t* ref, const uint16_t* cur, int32_t Hp, int32_t Wp,
                            int32_t B, int32_t R, int32_t step, const int16_t* pred, int32_t limit,
                            const int32_t* blocks, int32_t n_blocks,
                            int16_t* mv, int32_t* sad, int64_t* ops_valid, int64_t* ops_enum,
                            int32_t nthreads)
{
    if (Hp <= 0 || Wp <= 0 || B <= 0 || R < 0 || step <= 0 || limit < 0) return -1;
    const int32_t bh = (Hp + B - 1) / B, bw = (Wp + B - 1) / B;
    const int32_t nb = blocks ? n_blocks : bh * bw;
    int64_t tot_valid = 0, tot_enum = 0;
    int32_t overflow = 0;
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tot_valid, tot_enum) reduction(| : overflow) num_threads(nt)
    for (int32_t t = 0; t < nb; ++t) {
        const int32_t b = blocks ? blocks[t] : t;
        const int32_t bi = b / bw, bj = b % bw;
        const int32_t y0 = bi * B, y1 = (y0 + B < Hp) ? y0 + B : Hp;
        const int32_t x0 = bj * B, x1 = (x0 + B < Wp) ? x0 + B : Wp;
        const int64_t samples = 4LL * (y1 - y0) * (x1 - x0);
        const int32_t px = pred ? pred[2 * b + 0] : 0;
        const int32_t py = pred ? pred[2 * b + 1] : 0;
        int have = 0;
        int64_t best_s = 0;
        int32_t best_dx = 0, best_dy = 0;
        for (int32_t v = -R; v <= R; ++v)
            for (int32_t u = -R; u <= R; ++u) {
                const int32_t dx = px + step * u, dy = py + step * v;
                tot_enum += samples;
                if (dx < -limit || dx > limit || dy < -limit || dy > limit) continue;
                if (y0 + dy < 0 || y1 + dy > Hp || x0 + dx < 0 || x1 + dx > Wp) continue;
                const int64_t s = block_sad(ref, cur, Hp, Wp, y0, y1, x0, x1, dx, dy);
                tot_valid += samples;
                if (!have || key_less(s, dx, dy, best_s, best_dx, best_dy)) {
                    have = 1;
                    best_s = s;
                    best_dx = dx;
                    best_dy = dy;
                }
            }
        if (have && best_s > INT32_MAX) overflow |= 1;
        mv[2 * b + 0] = (int16_t)(have ? best_dx : 0);
        mv[2 * b + 1] = (int16_t)(have ? best_dy : 0);
        sad[b] = have ? (int32_t)best_s : -1;
    }
    if (ops_valid) *ops_valid = tot_valid;
    if (ops_enum) *ops_enum = tot_enum;
    return overflow ? -2 : 0;
}

/* Full search (paper Sec. 2.2): predictor 0, step 1, limit R. */
int32_t oracle_full_search(const uint16_t* ref_mosaic, const uint16_t* cur_mosaic, int32_t H, int32_t W,
                           int64_t pitch_ref, int64_t pitch_cur, int32_t B, int32_t R,
                           const int32_t* blocks, int32_t n_blocks,
                           int16_t* mv, int32_t* sad, int64_t* ops_valid, int32_t nthreads)
{
    if (H <= 0 || W <= 0 || (H & 1) || (W & 1)) return -1;
    const int32_t Hp = H / 2, Wp = W / 2;
    uint16_t* rp = (uint16_t*)malloc(sizeof(uint16_t) * 4 * (size_t)Hp * Wp);
    uint16_t* cp = (uint16_t*)malloc(sizeof(uint16_t) * 4 * (size_t)Hp * Wp);
    if (!rp || !cp) {
        free(rp);
        free(cp);
        return -3;
    }
    oracle_pack_planes(ref_mosaic, H, W, pitch_ref, rp);
    oracle_pack_planes(cur_mosaic, H, W, pitch_cur, cp);
    int32_t rc = oracle_stage_search(rp, cp, Hp, Wp, B, R, 1, NULL, R, blocks, n_blocks, mv, sad, ops_valid, NULL,
                                     nthreads);
    free(rp);
    free(cp);
    return rc;
}
