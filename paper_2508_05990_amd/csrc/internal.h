// Internal declarations shared by the HIP sources of the library (not part of
// the public ABI, which is include/me.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

// Device pointers of one pair of a batch launch.
struct JobPtrs {
    const uint32_t* ref;
    const uint32_t* cur;
    int16_t* mv;
    int32_t* sad;
};

// One block-matching stage over one frame pair.  Frames are read as 32-bit
// words: word k of mosaic row r holds samples (r, 2k) and (r, 2k+1), i.e. the
// packed-plane pixel column k of the two planes that live on row r's parity.
// A packed displacement (dx, dy) is then a displacement of dx words and 2*dy
// mosaic rows.
// One frame pair of a queue launch (batch submission): its pointers, geometry,
// radius and window plan.  A launch's items are the (block row, block group)
// pairs of every job's full-width blocks, job after job; item0 is the job's
// first item.
struct QueueJob {
    const uint32_t* ref;
    const uint32_t* cur;
    int16_t* mv;
    int32_t* sad;
    int64_t ref_pitch, cur_pitch;   // words per mosaic row
    int32_t Hp, Wp, bh, bw;
    int32_t R;
    int32_t nb, wpb;                // blocks per item, waves per block
    int32_t band_ty, lds_pitch, cur_lds;
    int32_t cols;                   // full-width block columns
    int32_t groups;                 // items per block row, ceil(cols / nb)
    int32_t item0;
    int32_t rs;                     // remainder rows as single candidates
};

struct QueueArgs {
    const QueueJob* jobs;           // device table, ordered by item0
    int32_t n_jobs;
    int32_t n_items;
    int32_t* counter;               // zero at launch; the launch leaves it zero
};

struct SearchArgs {
    const uint32_t* ref;
    const uint32_t* cur;
    int64_t ref_pitch;      // words per mosaic row
    int64_t cur_pitch;
    int32_t block;          // B, packed pixels (8, 16, 32, 64)
    int32_t Hp, Wp;         // packed plane size
    int32_t bh, bw;         // block grid
    int32_t R;              // candidates per side around the predictor
    int32_t limit;          // |dx|, |dy| <= limit
    const int16_t* pred;    // [bh/pred_ratio][pred_bw][2] or null (predictor 0)
    int32_t pred_ratio;     // block (bi, bj) takes the predictor of (bi/ratio, bj/ratio)
    int32_t pred_bw;        // row length of pred
    int32_t step;           // candidates p + step * (u, v)
    const int32_t* list;    // optional block list (device); null = all blocks
    const int32_t* list_n;  // device count for `list` (blocks past it exit)
    int16_t* mv;            // [bh][bw][2]
    int32_t* sad;           // [bh][bw]
    int32_t band_ty;        // candidate tile rows per LDS band
    int32_t lds_pitch;      // words per LDS window row (multiple of 4)
    int32_t col0, ncols;    // block columns covered by a launch without a list
    int32_t nb;             // horizontally adjacent blocks per workgroup (1 with a list or predictors)
    int32_t cur_lds;        // LDS word offset of the staged current blocks (shapes with cl = 1)
    int32_t wpb;            // waves per block of the tiled kernel (nb * wpb waves per workgroup)
    int32_t rs;             // remainder rows as single candidates (TileCfg::rs)
    // batch launch: n_jobs pairs of this shape (block, radius, frame size,
    // pitches); each workgroup takes ref/cur/mv/sad of its pair from jobs[]
    // instead of the fields above.  Null for a single pair.
    const JobPtrs* jobs;
    int32_t n_jobs;
    // proposal refine (small-radius kernel only): predictors decoded from the
    // network output [3][bh][bw], clamp(rint(8 o), -limit, limit), instead of
    // `pred`; null otherwise
    const float* net;
    // fused warp (tiled and generic kernels, single pair): once a block's
    // vector is known, its workgroup also writes the block's cells of
    // wout = Warp(wz, MV) ([wC][wHf][wWf], cell size ws packed pixels, float32
    // or bfloat16).  wz null: no warp.
    const void* wz;
    void* wout;
    int32_t wC, wHf, wWf, ws, wbf16;
    float winv_s;
};


// Launch shape of the search kernel.
struct TileCfg {
    int kx;        // horizontally adjacent candidates per lane
    int ky;        // vertically adjacent candidates per lane
    int nb;        // blocks per workgroup (4 waves each)
    int band_ty;   // tile rows per LDS band
    int lds_pitch; // words per LDS row
    size_t lds_bytes;
    int cl;        // 1: current blocks staged in LDS (after the window); 0: read through scalar loads
    int wpb;       // waves per block: 2, 4 or 8 (0 = 4)
    int rs;        // 1: candidate rows below the main tiles as single candidates (else KX x 1 tiles)
};

// Fill in the LDS geometry of `cfg` (kx, ky, nb set) for block size B and
// radius R; band_ty is the largest that keeps the window within lds_cap
// bytes.  Returns false if no band fits.
bool plan_tiles(int B, int R, size_t lds_cap, TileCfg* cfg);

// Default launch shape for block size B and radius R.
TileCfg default_tiles(int B, int R);

// Launch shape of the full search over a device block list (one block per
// workgroup).
TileCfg list_tiles(int B, int R);

// Whether the kernel table has an instance for (B, kx, ky).
bool tiles_supported(int B, int kx, int ky);

// Whether a stage search with step > 1 fits the strided kernel's LDS plan.
bool step_supported(int B, int R, int step);

// Whether a search of radius R takes the small-radius kernel (the only one
// that accepts a.net, the fused proposal decode).
bool small_search(int B, int R);

// Full or stage search of one pair, of a.n_jobs pairs of one shape
// (a.jobs), or of the first *a.list_n blocks of a.list (n_wg = list capacity).
// parts: 1 = full-width blocks (tiled kernel), 2 = blocks cut by the right
// frame edge (generic kernel), 3 = both.
hipError_t launch_sad_search(const SearchArgs& a, const TileCfg& cfg, int n_wg, hipStream_t stream, int parts = 3);

// Queue launches (batch submission): tile shapes with a queue kernel; the
// plan of one job for the launch's tile (kx, ky, cl) within lds_cap bytes
// (fills nb, wpb, band_ty, lds_pitch, cur_lds, cols, groups; the caller sets
// item0), and the launch over all jobs of one block size (lds_bytes: the
// largest job plan).
bool queue_supported(int B, int kx, int ky);
bool plan_queue_job(int B, const TileCfg& tile, size_t lds_cap, QueueJob* j, size_t* lds_bytes);
hipError_t launch_sad_queue(const QueueArgs& q, int B, const TileCfg& tile, size_t lds_bytes, hipStream_t stream);

// Chained block vectors over a group of pictures (out may alias ms).
hipError_t launch_compose(const int16_t* ms, const int16_t* ma, int16_t* out, int bh, int bw, int B, int Hp, int Wp,
                          hipStream_t stream);

// Bilinear propagation of a feature map by block vectors.
hipError_t launch_warp(const void* z, void* out, int bf16, int C, int Hf, int Wf, const int16_t* mv, int bw,
                       int cells, int s, hipStream_t stream);

// Learned-proposal refine/fallback helpers (refine.hip).
hipError_t launch_decode(const float* out, int nblk, int R, int16_t* pred, hipStream_t stream);
hipError_t launch_fallback(const float* out, const int32_t* sad, int bh, int bw, int Hp, int Wp, int B,
                           float conf_thresh, double ratio_m, uint8_t* fb, int32_t* list, int32_t* count,
                           hipStream_t stream);

// Proposal network (cnn.hip).  Layer l = 0..3: (cin, cout, stride) =
// (8,32,2), (32,32,2), (32,32,1), (32,3,1).
constexpr int kCnnParams = 21699;
int cnn_fwd_packed_size(int l);
int cnn_bwd_packed_size(int l);
int cnn_wgrad_groups(int n, int Ho, int Wo);
size_t cnn_wgrad_partial_floats(int l, int nwg);
hipError_t launch_pool(const uint16_t* ref, int64_t ref_pitch, const uint16_t* cur, int64_t cur_pitch, int Hq, int Wq,
                       uint16_t* out, hipStream_t st);
hipError_t launch_pack(const float* w, uint16_t* fwd, uint16_t* bwd, hipStream_t st);
hipError_t launch_conv_fwd(int l, const uint16_t* in, const uint16_t* wp, const float* bias, void* out, int n, int H,
                           int W, int Ho, int Wo, hipStream_t st);
// The four layers in one launch for inference (activations in LDS); the same
// products in the same order as conv_fwd_kernel, so the same bits.  a0..a2
// (optional, all or none) receive the layer 0..2 activations.
hipError_t launch_cnn_fused(const uint16_t* in, const uint16_t* wf, const float* params, float* out, int n, int Hq,
                            int Wq, uint16_t* a0, uint16_t* a1, uint16_t* a2, hipStream_t st);
hipError_t launch_loss(const float* out, const int16_t* mv, const float* wt, int n, int nblk, int R, int rr,
                       uint16_t* dz, float* bl, float* loss, hipStream_t st);
hipError_t launch_conv_dgrad(int l, const uint16_t* dz, const uint16_t* wb, const uint16_t* aprev, uint16_t* dprev,
                             int n, int H, int W, int Ho, int Wo, hipStream_t st);
hipError_t launch_conv_wgrad(int l, const uint16_t* x, const uint16_t* dz, float* partial, float* grads, int n, int H,
                             int W, int Ho, int Wo, hipStream_t st);
hipError_t launch_adamw(float* w, const float* g, float* m, float* v, int np, float lr, float b1, float b2, float eps,
                        float wd, float c1, float c2, hipStream_t st);

// Perception residual network (prnet.hip).  A tensor view: pixel p = (n, y, x)
// of HW pixels per image, C channels (a multiple of 4), stored [n][HW][C]
// (chw = 0) or [n][C][HW] (chw = 1), float32 (f32 = 1) or bfloat16.
struct PwTensor {
    const void* p;
    int32_t C, chw, f32;
};

// 1x1 convolution (or its input gradient) as a GEMM over P pixels: out[p][m]
// = sum_k A[m][k] x[p][k] with x = [x, x2] along k; then + bias, ReLU6, + add,
// times the ReLU6 derivative of mask (bfloat16 [P][M]); stored as `out`.
struct PwArgs {
    PwTensor x, x2;             // x2.p may be null
    int32_t HW, P;
    const uint16_t* w;          // packed A operand, (M/16 rounded up) x KS tiles
    int32_t M, KS;              // output channels (multiple of 4), K / 16
    const float* bias;          // [M] or null
    int32_t relu6;
    PwTensor add;               // add.p may be null; add.C == M
    const uint16_t* mask;       // or null
    void* out;
    int32_t out_chw, out_f32;
};

// Weight gradient of a 1x1 convolution: dW[o][c] = sum_p dy[p][o] x[p][c],
// db[o] = sum_p dy[p][o]; per-workgroup partials (chunk pixels each) then a
// fixed-order reduction.
struct PwGradArgs {
    PwTensor x, x2, dy;
    int32_t HW, P, cin, cout, chunk;
    float* partial;             // nwg * (cout * cin + cout) floats
};

size_t pw_lds_bytes(int KS);
size_t pw_wgrad_lds_bytes(int cin, int cout);
int wgrad_chunk(int P, int target_wg);
hipError_t launch_pw(const PwArgs& a, hipStream_t st);
hipError_t launch_pw_pack(const float* w, int ld, int m0, int trans, int Mv, int Kv, int MT, int KS, uint16_t* out,
                          hipStream_t st);
hipError_t launch_pw_wgrad(const PwGradArgs& a, float* gw, float* gb, hipStream_t st);
hipError_t launch_dw_fwd(const uint16_t* x, const float* w, const float* b, uint16_t* y, int n, int H, int W, int C,
                         int S, int relu6, hipStream_t st);
hipError_t launch_dw_dgrad(const uint16_t* dy, const float* w, const uint16_t* mask, uint16_t* dx, int n, int H, int W,
                           int C, int S, hipStream_t st);
int dw_wgrad_nwg(int n, int Ho, int Wo);   // workgroups (partial rows) of a depthwise weight gradient
hipError_t launch_dw_wgrad(const uint16_t* x, const uint16_t* dy, float* partial, float* gw, float* gb, int n, int H,
                           int W, int C, int S, hipStream_t st);
hipError_t launch_planes(const uint16_t* m, int64_t pitch, int64_t img_stride, int n, int Hp, int Wp, uint16_t* out,
                         hipStream_t st);
// One inverted residual block fused (inference): h_out = h + Wc ReLU6(dw(ReLU6(We h + be)) + bd) + bc,
// activations bfloat16 channels-last [n][Hf][Wf][ch]; we / wc: packed A operands of the expansion
// (m = x, k = ch) and compression (m = ch, k = x); wd float32 [x][9].
struct IrArgs {
    const uint16_t* h_in;
    uint16_t* h_out;
    const uint16_t* we;
    const float* be;
    const float* wd;
    const float* bd;
    const uint16_t* wc;
    const float* bc;
    int32_t n, Hf, Wf, ch, x;
};
bool ir_fused_ok(int ch, int x);

// The encoder fused (inference): packed planes of the mosaic, depthwise s2 +
// ReLU6 (4 channels), 1x1 4 -> ce + ReLU6, depthwise s2 + ReLU6, 1x1 ce -> ce
// + ReLU6, written as bfloat16 channels-last [n][Hf][Wf][ce].  Float32 master
// parameters of the four layers; w3p: packed A operand of the last 1x1.
struct EncArgs {
    const uint16_t* mosaic;
    int64_t pitch, img_stride;
    int32_t n, Hp, Wp, H1, W1, Hf, Wf, ce;
    const float *w0, *b0, *w1, *b1, *w2, *b2, *b3;
    const uint16_t* w3p;
    uint16_t* out;
};
bool enc_fused_ok(int ce);
hipError_t launch_encoder(const EncArgs& a, hipStream_t st);
hipError_t launch_ir_block(const IrArgs& a, hipStream_t st);
hipError_t launch_to_nhwc(const void* src, int f32, int n, int C, int HW, uint16_t* dst, hipStream_t st);
int prloss_blocks(int P);
hipError_t launch_prloss(const float* r, const float* zp, const float* zt, int n, int C, int HW, float tau,
                         int32_t* nbad, uint32_t* maxbits, uint8_t* flags, uint16_t* dr, float* partial, float* loss,
                         hipStream_t st);

// Training-set statistics (stats.hip): lower median of the per-sample SAD of
// N = n * nblk blocks (hist: 256 counters, state: 2 words of scratch), and the
// 0/1 weight sad <= floor(ratio_m * n_samples).
hipError_t launch_sad_median(const int32_t* sad, int64_t N, int nblk, int bw, int Hp, int Wp, int B, uint32_t* hist,
                             uint32_t* state, float* median, hipStream_t st);
hipError_t launch_fallback_weight(const int32_t* sad, int64_t N, int nblk, int bw, int Hp, int Wp, int B,
                                  double ratio_m, float* weight, hipStream_t st);

hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t stream);
hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t stream);

}  // namespace me
