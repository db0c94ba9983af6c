/*
 * me.h -- C ABI of the MI355X Bayer-domain motion-estimation library.
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the data-parallel
 * hot path of "Efficient Bayer-Domain Video Computer Vision with Fast Motion
 * Estimation and Learned Perception Residual" (arXiv 2508.05990):
 *
 *   MV     = ME(F_R, F_C)        block-matching motion estimation with the SAD
 *                                criterion on raw Bayer frames (paper Sec. 2.2
 *                                "Definition", Sec. 3.2 "Matching Criterion");
 *   z_pred = Warp(z_R, MV)       propagation of the reference frame's feature
 *                                map by the block vectors (paper Sec. 3.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.  Every data pointer is a DEVICE pointer owned by the caller unless
 *   the comment says "host".  The library never frees a caller pointer and
 *   does not keep it past the stream work of the call.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Work is enqueued asynchronously; nothing is synchronised.
 * Errors.  Arguments are validated before any device work, and a failed
 *   validation enqueues nothing.  Launch failures return ME_E_HIP.  Faults of
 *   the asynchronous work itself surface from the next synchronising HIP call.
 *   me_last_error() gives a readable message for the calling thread's last
 *   failure.  No C++ exception crosses this interface.
 * Frames.  A frame is a Bayer mosaic of uint16 samples, RGGB at (0,0): R at
 *   even row/even column, Gr at even/odd, Gb at odd/even, B at odd/odd.  The
 *   search works on the four packed colour planes
 *   P[c][y][x] = M[2y + (c>>1)][2x + (c&1)] (Hp = H/2 rows, Wp = W/2 columns),
 *   read straight from the mosaic.  Sizes, radii and vectors are in packed
 *   pixels (one packed pixel = two Bayer pixels in each direction).
 * Blocks.  Block (i, j) covers packed rows [iB, min(iB+B, Hp)) and columns
 *   [jB, min(jB+B, Wp)); the last row/column of blocks may be partial.
 *   bh = ceil(Hp/B), bw = ceil(Wp/B).  Per-block outputs are row-major
 *   [bh][bw].
 * Vectors.  mv[b] = (dx, dy), int16, the position of the best match in the
 *   reference frame minus the block's position in the current frame (a scene
 *   translated by +s between reference and current gives -s).
 * Selection.  Lowest SAD over the four planes (paper Sec. 3.2); ties go to the
 *   smaller dx*dx+dy*dy, then the smaller dy, then the smaller dx, so the
 *   result is unique.  Only candidates whose displaced block lies wholly
 *   inside the reference frame are considered.
 * Threads.  A context is not thread-safe; separate contexts are independent.
 */
#ifndef ME_H
#define ME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ME_OK = 0,
    ME_E_INVAL = 1,        /* bad argument: null pointer, bad size, inconsistent geometry */
    ME_E_UNSUPPORTED = 2,  /* valid request the library does not implement (e.g. B=12) */
    ME_E_HIP = 3,          /* a HIP runtime call failed (no device, launch failure) */
    ME_E_NOMEM = 4,        /* device or host allocation failed */
    ME_E_STATE = 5         /* call not valid in the context's state (e.g. no weights loaded) */
} me_status;

typedef enum { ME_MODE_EXHAUSTIVE = 0, ME_MODE_PROPOSAL = 1 } me_mode;
typedef enum { ME_F32 = 0, ME_BF16 = 1 } me_dtype;

typedef struct me_ctx_s* me_ctx;

/* A Bayer frame in device memory.  height and width (Bayer samples) are even
 * and at least 2; pitch (elements between rows) is even and >= width; data is
 * 4-byte aligned.  Samples are used as unsigned 16-bit values. */
typedef struct {
    const uint16_t* data;
    int32_t height;
    int32_t width;
    int64_t pitch;
} me_frame;

typedef struct {
    int32_t block;                 /* B, packed pixels: 8, 16, 32 or 64 */
    int32_t radius;                /* R, candidates per side: 1..64 (full search: (2R+1)^2 candidates) */
    int32_t step;                  /* candidate spacing; me_estimate takes 1 (me_stage_search any) */
    int32_t mode;                  /* me_mode */
    int32_t refine_radius;         /* proposal mode: exact search radius around the proposal (0..8) */
    float conf_logit_thresh;       /* proposal mode: fall back when logit < this (0 <=> confidence 0.5) */
    float sad_ratio;               /* proposal mode: fall back when SAD > floor(ratio * M * n) */
    float sad_median_per_sample;   /* proposal mode: M; <= 0 selects the value loaded with the weights */
} me_params;

/* Default parameters: B=16, R=32, step 1, exhaustive, refine radius 2,
 * logit threshold 0, SAD ratio 1.5, median from the weights. */
me_params me_default_params(void);

/* Create a context on HIP device `device`.  Contexts own scratch buffers,
 * loaded proposal weights and captured graphs.  *out is set on success. */
me_status me_ctx_create(int32_t device, me_ctx* out);
me_status me_ctx_destroy(me_ctx ctx);

/*
 * me_estimate -- MV = ME(F_R, F_C) (paper Sec. 2.2; Sec. 3.2 SAD criterion;
 * full search of Sec. 2.2 in ME_MODE_EXHAUSTIVE).
 *
 * ref, cur : host structs describing device frames of equal height/width.
 * params   : host struct; see me_params.
 * mv       : device, int16 [bh][bw][2] (dx, dy), written.
 * sad      : device, int32 [bh][bw], SAD of the chosen vector, written.
 * fallback : device, uint8 [bh][bw] or NULL; in proposal mode 1 where the
 *            block fell back to full search, 0 otherwise (all 0 in
 *            exhaustive mode).
 * ctx may be NULL in exhaustive mode (no state is needed); proposal mode
 * needs a context with weights loaded (ME_E_STATE otherwise).
 */
me_status me_estimate(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params* params,
                      int16_t* mv, int32_t* sad, uint8_t* fallback, void* stream);

/*
 * me_stage_search -- one block-matching stage around per-block predictors
 * (paper Sec. 3.2: one matching stage evaluates a set of candidates per
 * block with one thread group per block; its coarse, intermediate and fine
 * stages differ in range and step).  Candidates are p + step * (u, v) with
 * u, v in [-radius, radius]; a candidate is kept if the displaced block is
 * inside the reference frame and |dx|, |dy| <= limit.
 *
 * pred : device int16 [bh][bw][2] (dx, dy), or NULL for p = 0.
 * step : >= 1; step > 1 needs block + 2 radius step <= 256 (ME_E_UNSUPPORTED
 *        otherwise).
 * limit: 0..127.
 * A block with no valid candidate gets sad = -1 and mv = (0, 0).
 * ctx may be NULL.
 */
me_status me_stage_search(me_ctx ctx, const me_frame* ref, const me_frame* cur, int32_t block, int32_t radius,
                          int32_t step, const int16_t* pred, int32_t limit, int16_t* mv, int32_t* sad,
                          void* stream);

/* Block pyramid and stages of me_pyramid. */
typedef struct {
    int32_t n_levels;      /* 1..4 */
    int32_t block[4];      /* packed pixels per level, coarse to fine; each in
                              {8,16,32,64} and dividing the previous one */
    int32_t n_stages;      /* 1..4 stages per level */
    int32_t radius[4];     /* per stage, 0..64 */
    int32_t step[4];       /* per stage, >= 1 */
    int32_t limit;         /* |dx|, |dy| <= limit for every candidate, 0..127 */
} me_pyramid_cfg;

/* The paper's standard setting (FME settings table of Sec. 4): blocks of 64
 * and 32 Bayer pixels (32 and 16 packed pixels), stages (range, step) =
 * (8, 8), (4, 4), (2, 1), limit 127. */
me_pyramid_cfg me_default_pyramid(void);

/*
 * me_pyramid -- coarse-to-fine block matching over a block pyramid (paper
 * Sec. 3.2, "Pyramid Block Structure" and "Parallel Coarse-to-fine Block
 * Matching").  Levels run from the largest block to the smallest; each runs
 * its stages in order, each a stage search around the previous stage's
 * vectors; the first stage of the first level starts from zero, that of a
 * finer level from the vector of the coarser block containing each block.
 * mv / sad: device [bh][bw] of the finest level's block grid.  Needs a
 * context (intermediate vectors live in its scratch).
 */
me_status me_pyramid(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_pyramid_cfg* cfg, int16_t* mv,
                     int32_t* sad, void* stream);

/*
 * me_warp_features -- z_pred = Warp(z_R, MV) (paper Sec. 3.3).
 *
 * z_ref : device [C][Hf][Wf], float32 or bfloat16 (dtype), contiguous.
 * z_out : device, same type and shape, written; must not overlap z_ref.
 * mv    : device int16 [bh][bw][2] from me_estimate with the same block size
 *         on a frame of frame_h x frame_w Bayer samples.
 * Geometry: s = (frame_h/2)/Hf must equal (frame_w/2)/Wf, be a whole number
 * and divide `block` (ME_E_UNSUPPORTED otherwise).  Cell (i, j) lies in block
 * (i*s/B, j*s/B); with that block's (dx, dy) the output is the bilinear
 * sample of z_ref at (i + dy/s, j + dx/s), the two row and two column indices
 * clamped into the map.  Float32 arithmetic; bfloat16 inputs are widened and
 * the result is rounded to nearest even.
 * ctx may be NULL.
 */
me_status me_warp_features(me_ctx ctx, const void* z_ref, void* z_out, int32_t dtype, int32_t C, int32_t Hf,
                           int32_t Wf, const int16_t* mv, int32_t block, int32_t frame_h, int32_t frame_w,
                           void* stream);

/*
 * me_estimate_warp -- me_estimate (exhaustive, step 1) and me_warp_features in
 * one pass: each workgroup of the search, once its blocks' vectors are known,
 * writes those blocks' cells of z_out = Warp(z_ref, MV) (paper Sec. 3.3), so
 * the warp's memory traffic overlaps the search's integer work and needs no
 * second launch.  Arguments as in me_estimate (mv, sad written) and
 * me_warp_features (z_ref, z_out, dtype, C, Hf, Wf; the map tiles the packed
 * frame with square cells that divide the block; z_out may not overlap z_ref).
 * Results are bit-identical to me_estimate followed by me_warp_features.
 * Radii served by the small-radius kernel (<= 4) run the two kernels in turn.
 */
me_status me_estimate_warp(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params* params, int16_t* mv,
                           int32_t* sad, const void* z_ref, void* z_out, int32_t dtype, int32_t C, int32_t Hf,
                           int32_t Wf, void* stream);

/*
 * me_compose_vectors -- chain block vectors over a group of pictures (paper
 * Sec. 4.1 GOP test protocol; Sec. 4.4 compares references).  mv_step maps the
 * blocks of frame t to frame t-1, mv_acc_in the blocks of frame t-1 to the key
 * frame; mv_acc_out[b] = mv_step[b] + mv_acc_in[b'], where b' is the block of
 * frame t-1 containing block b's centre (x0 + w/2, y0 + h/2) displaced by
 * mv_step[b] (block indices clamped to the grid).  All device int16
 * [bh][bw][2] for `block` on a frame_h x frame_w mosaic; sums wrap to int16.
 * mv_acc_out may alias mv_step but not mv_acc_in.
 */
me_status me_compose_vectors(const int16_t* mv_step, const int16_t* mv_acc_in, int16_t* mv_acc_out, int32_t block,
                             int32_t frame_h, int32_t frame_w, void* stream);

/*
 * me_refine -- refine-and-fallback step of the learned-proposal mode, given
 * the proposal network's per-block output.  The proposal network is this
 * library's addition: the paper's own learned part corrects features
 * (Sec. 3.3), not vectors.  The selection rule is still the paper's lowest
 * SAD (Sec. 3.2) over an exact search, so every output vector is either the
 * exact result of a small search around the proposal or the full-search
 * result.
 *
 * net_out : device float32 [3][bh][bw]: mvx, mvy (units of 8 packed pixels)
 *           and a confidence logit, per block.
 * Steps   : p = clamp(rint(8*o), -radius, radius) (ties to even); exact
 *           search of radius params->refine_radius around p, candidates
 *           limited to |dx|, |dy| <= radius; fallback to full search of
 *           params->radius when logit < conf_logit_thresh, or the refined
 *           SAD > floor(sad_ratio * M * n) (n = samples in the block, M =
 *           sad_median_per_sample or, if that is <= 0, the value loaded with
 *           the weights; the product is taken in double, left to right), or
 *           the refine window has no valid candidate.
 * mv, sad : device outputs as in me_estimate; fallback: device uint8
 *           [bh][bw] or NULL (1 = fell back).
 * Needs a context (scratch buffers live there); ME_E_STATE if no M is known.
 */
me_status me_refine(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params* params,
                    const float* net_out, int16_t* mv, int32_t* sad, uint8_t* fallback, void* stream);

/*
 * me_refine_noalloc -- me_refine for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, steps, kernels and results (bit for bit)
 * as me_refine, but the step's scratch (decoded proposals, fallback flags,
 * the fallback list and its count) lives in a fixed device array of the
 * library, 9 * ME_NOALLOC_MAX_BLOCKS + 256 bytes (576 KiB) on each device the
 * library runs on, held until the process ends, instead of context buffers
 * grown with hipMalloc.  The call allocates nothing, host or device.
 *   - ME_E_INVAL if the frame has more than ME_NOALLOC_MAX_BLOCKS blocks
 *     (checked before the context), and for the arguments me_refine rejects.
 *   - The array's address is resolved by me_ctx_create for the context's
 *     device; kernels run on `stream`, which must belong to that device.
 *   - Every call on one device shares that device's array and leaves the last
 *     call's contents in it (each call rewrites the count and the list it
 *     reads): calls that overlap on one device -- different streams, host
 *     threads or contexts without ordering between them -- race.  Order them
 *     on one stream.
 */
#define ME_NOALLOC_MAX_BLOCKS 65536
me_status me_refine_noalloc(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params* params,
                            const float* net_out, int16_t* mv, int32_t* sad, uint8_t* fallback, void* stream);

/*
 * Proposal network (learned-proposal mode; this library's addition, see
 * me_refine).  Input: for a frame pair of H x W Bayer samples (H, W divisible
 * by 8), the 4x4 means of each of the four packed planes of the reference
 * (channels 0-3) and current frame (4-7) -- the packed pair at a quarter of its
 * resolution per axis -- normalised to (v - 2048) / 1024, bfloat16, channels
 * last [H/8][W/8][8].  Four 3x3 convolutions, zero padding 1,
 * strides 2, 2, 1, 1, channels 8 -> 32 -> 32 -> 32 -> 3, ReLU after the first
 * three, bfloat16 weights and activations with float32 accumulation (MFMA);
 * output float32 [3][bh][bw] per pair for 16x16 blocks: mvx, mvy (units of 8
 * packed pixels) and a confidence logit.  Training loss: mean over blocks of
 * the reverse Huber (BerHu, paper Sec. 3.3) of each vector component against
 * full-search vector / 8 (threshold 1, i.e. 8 packed pixels), plus the binary cross-entropy of
 * the logit against "the full-search vector lies within refine_radius of the
 * decoded proposal"; AdamW (beta 0.9/0.999, eps 1e-8, weight decay 0.01) as
 * in the paper's training details (Sec. 4.1).
 *
 * Parameters: ME_CNN_NPARAMS float32 values, per layer W[out][in][3][3] then
 * b[out], layers in order.  Activations between layers are bfloat16
 * channels-last [n][h][w][32]; the output of layer 3 is float32
 * [n][3][bh][bw].  Device buffers passed to these calls are 16-byte aligned.
 */
#define ME_CNN_NPARAMS 21699

/* Set the master parameters (host array) and the median per-sample SAD used
 * by the fallback test; resets the optimiser state.  Synchronous. */
me_status me_cnn_set_params(me_ctx ctx, const float* params, int32_t count, float median_per_sample);
/* Copy the master parameters (and median, if not NULL) to host memory.  Synchronous. */
me_status me_cnn_get_params(me_ctx ctx, float* params, int32_t count, float* median_per_sample);
/* Network input of one frame pair into x (device bfloat16 [H/8][W/8][8]). */
me_status me_cnn_pool(me_ctx ctx, const me_frame* ref, const me_frame* cur, uint16_t* x, void* stream);
/* Forward of n pooled inputs x ([n][Hq][Wq][8]) into out (device float32 [n][3][bh][bw]),
 * all four layers in one launch with the activations in LDS (the path
 * me_estimate's proposal mode takes).  Each output takes its products in the
 * order of the layer-by-layer kernels of the training step, so the two agree
 * bit for bit.
 * me_cnn_forward_acts: the same launch, also storing the activations of
 * layers 0, 1, 2 (device bfloat16 [n][h1][w1][32], [n][h2][w2][32],
 * [n][h2][w2][32]; h1 = ceil(Hq/2), h2 = ceil(h1/2), 16-byte aligned) for
 * checking each layer on its own. */
me_status me_cnn_forward(me_ctx ctx, const uint16_t* x, int32_t n, int32_t Hq, int32_t Wq, float* out, void* stream);
me_status me_cnn_forward_acts(me_ctx ctx, const uint16_t* x, int32_t n, int32_t Hq, int32_t Wq, float* out,
                              uint16_t* a0, uint16_t* a1, uint16_t* a2, void* stream);
/*
 * One training step on n pooled inputs and their full-search vectors mv
 * (device int16 [n][bh][bw][2]): forward, loss (mean over the n x bh x bw
 * blocks of w x (BerHu of the two vector components) + BCE of the confidence
 * logit, Sec. 3.3 loss family), backward; with update != 0 an AdamW step with
 * learning rate lr.  weight (device float32 [n][bh][bw], NULL = all 1) is the
 * per-block weight w of the vector term, e.g. 0 for blocks whose full-search
 * match is too poor for a proposal ever to be accepted.  grads (device
 * float32 [ME_CNN_NPARAMS]) and loss (device float32 scalar) receive the
 * gradient and loss when not NULL.  Weight gradients are reduced in a fixed
 * order: the same inputs give bit-identical results.
 */
me_status me_cnn_train_step(me_ctx ctx, const uint16_t* x, const int16_t* mv, const float* weight, int32_t n,
                            int32_t Hq, int32_t Wq, int32_t radius, int32_t refine_radius, float lr, int32_t update,
                            float* grads, float* loss, void* stream);
/* Checkpoint of the optimiser state (parameters, both moments, step count,
 * median) in a host buffer of me_cnn_state_bytes() bytes.  Synchronous. */
int64_t me_cnn_state_bytes(void);
me_status me_cnn_save_state(me_ctx ctx, void* buf, int64_t bytes);
me_status me_cnn_load_state(me_ctx ctx, const void* buf, int64_t bytes);
/* Single stages, for checking each kernel on its own: layer `layer` (0..3)
 * forward of a [n][H][W][cin] input; its backward given the layer input x and
 * the gradient dz of its output ([n][Ho][Wo][coutp], coutp = 32, or 4 for
 * layer 3 with channel 3 zero), writing the layer's slice of grads and, for
 * layer > 0, the input gradient masked by the input's ReLU (x > 0) into dx;
 * the loss of float32 outputs against labels (weight as for the training
 * step; dz: bfloat16 [n][nblk][4], loss: float32 scalar; synchronous); an AdamW step with given gradients. */
me_status me_cnn_layer_forward(me_ctx ctx, int32_t layer, const uint16_t* in, void* out, int32_t n, int32_t H,
                               int32_t W, void* stream);
me_status me_cnn_layer_backward(me_ctx ctx, int32_t layer, const uint16_t* x, const uint16_t* dz, uint16_t* dx,
                                float* grads, int32_t n, int32_t H, int32_t W, void* stream);
me_status me_cnn_loss(me_ctx ctx, const float* out, const int16_t* mv, const float* weight, int32_t n, int32_t nblk,
                      int32_t radius, int32_t refine_radius, uint16_t* dz, float* loss, void* stream);
me_status me_cnn_adamw(me_ctx ctx, const float* grads, float lr, void* stream);

/* One frame pair of a batch (me_batch_submit).  params.mode must be
 * ME_MODE_EXHAUSTIVE with step 1: a batch job has no fallback output and no
 * network state, so pairs in learned-proposal mode go through me_estimate
 * (ME_E_UNSUPPORTED otherwise). */
typedef struct {
    me_frame ref;
    me_frame cur;
    me_params params;      /* exhaustive mode, step 1 */
    int16_t* mv;           /* device [bh][bw][2] */
    int32_t* sad;          /* device [bh][bw] */
} me_job;

/*
 * me_batch_submit -- many independent frame pairs of mixed sizes, block sizes
 * and radii (the paper's batched grid over (Batch, h, w), Sec. 4.1 CUDA
 * settings, extended to uneven jobs).  jobs is a HOST array of n entries
 * (read before return); results are bit-identical to n separate me_estimate
 * calls.  All jobs of one block size go through ONE persistent launch: a
 * workgroup per resident slot repeatedly takes the next item -- a run of
 * horizontally adjacent full-width blocks of one job, with that job's own
 * radius, frame size and window plan -- from a device ticket counter until
 * none is left; jobs are ordered by decreasing work per item.  Blocks cut by
 * the right frame edge (frame width not a multiple of the block) are searched
 * by an extra launch per job shape.  The launches are captured once as one HIP
 * graph and replayed while the job shapes (block, radius, size, pitches, in
 * order) repeat; each submission restages the pairs' pointers into
 * context-owned device tables through pinned memory.  Submissions that use
 * one context share those tables and the ticket counters: on one stream they
 * are ordered; across streams the caller must order them (or use one context
 * per stream).  Returns ME_E_UNSUPPORTED for jobs other than exhaustive step 1.
 */
me_status me_batch_submit(me_ctx ctx, const me_job* jobs, int32_t n, void* stream);

/*
 * me_autotune -- time the candidate launch shapes of the full-search kernel
 * (candidate tile shape per lane, blocks per workgroup, LDS window band) on
 * this frame pair with HIP events and keep the fastest in the context for
 * (block, radius, frame size); later me_estimate calls with that key use it.
 * Every shape gives bit-identical results.  Synchronises `stream`; a batch
 * graph captured earlier in the context is dropped (the next me_batch_submit
 * records the tuned shapes).
 * best_ms (host, may be NULL) receives the fastest mean time of `iters` runs.
 */
me_status me_autotune(me_ctx ctx, const me_frame* ref, const me_frame* cur, int32_t block, int32_t radius,
                      int32_t iters, float* best_ms, void* stream);

/*
 * me_tuned_shape -- the launch shape the context uses for a full search with
 * (block, radius) on height x width Bayer frames (batch grid of Sec. 4.1):
 * shape[0] candidates per lane along x, shape[1] along y, shape[2] blocks per
 * workgroup, shape[3] the LDS window size in KB (rounded up), shape[4] where the
 * kernel reads the current block from: 0 scalar loads, 1 LDS (staged beside
 * the window), shape[5] waves per block (2, 4 or 8; blocks x waves <= 8).
 * shape holds 6 entries.  *tuned (may be
 * NULL) is 1 when the shape was recorded by me_autotune or
 * me_set_tuned_shape, 0 when it is the built-in default.  Host call, no GPU
 * work.  ME_E_INVAL on a null pointer, odd or empty frame or radius outside
 * [0, 64]; ME_E_UNSUPPORTED on a block size outside {8, 16, 32, 64}.
 *
 * me_set_tuned_shape -- record a shape in that form (for instance one that
 * me_tuned_shape reported in an earlier process, so that tuning persists):
 * shape[3] is the LDS budget in KB (window and, with shape[4] = 1, the staged
 * current blocks); the window band is the largest that fits
 * it, so a reported shape set back gives the same launch.  Results do not
 * depend on the shape.  ME_E_INVAL when shape[4] is not 0 or 1 or shape[5]
 * not 2, 4 or 8; ME_E_UNSUPPORTED when the tile is not compiled for the block
 * size, blocks per workgroup x waves per block exceeds 8, more than one block
 * per workgroup with radius % 4 != 0, or no band fits the budget (at most
 * 158 KB); the stored table is unchanged then.  Drops a batch graph captured earlier in the context, synchronising
 * the device first.
 */
me_status me_tuned_shape(me_ctx ctx, int32_t block, int32_t radius, int32_t height, int32_t width, int32_t* shape,
                         int32_t* tuned);
me_status me_set_tuned_shape(me_ctx ctx, int32_t block, int32_t radius, int32_t height, int32_t width,
                             const int32_t* shape);

/* ------------------------------------------------------------------------
 * Perception residual network (PRNet, paper Sec. 3.3): corrects propagated
 * features, z_out = z_pred + r with r = PRNet(current frame, z_pred), trained
 * on the residual z_C - z_pred with a region-weighted reverse Huber (BerHu)
 * loss.  The paper gives the parts but no widths; the network here:
 *   encoder: two depthwise-separable blocks over the current frame's packed
 *     planes ((v - 2048) / 1024): depthwise 3x3 stride 2 (+bias, ReLU6), then
 *     1x1 to c_enc channels (+bias, ReLU6); output on the feature grid
 *     Hf = ceil(Hp/4), Wf = ceil(Wp/4) (Hp, Wp = packed plane size);
 *   projection: 1x1 over [z_pred, encoder] to c_hid channels (+bias, ReLU6);
 *   n_blocks inverted residual blocks: 1x1 to expand*c_hid (+bias, ReLU6),
 *     depthwise 3x3 stride 1 (+bias, ReLU6), 1x1 back to c_hid (+bias), plus
 *     the block input;
 *   head: 1x1 to c_feat channels (+bias): the residual r.
 * Loss per feature position p (t = z_target - z_pred): p counts as wrongly
 * propagated when the channel mean of |t| exceeds tau; each of the two
 * regions carries half the loss (a region that is empty, or tau < 0, gives
 * the plain mean); the term is BerHu(r - t) / c_feat with threshold
 * c = 0.2 max |r - t| over the batch (held constant in the gradient).
 * Parameters are one float32 vector, layer by layer in the order above
 * (weights then biases; depthwise weights [C][9], tap = 3 ky + kx; 1x1
 * weights [c_out][c_in]).  Activations are bfloat16 channels-last; 1x1
 * convolutions run on bfloat16 MFMA with float32 accumulation; depthwise
 * weights and all biases stay float32.  Features are [n][c_feat][Hf][Wf].
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t c_feat;    /* feature channels, multiple of 16 */
    int32_t c_enc;     /* encoder channels, multiple of 16 */
    int32_t c_hid;     /* hidden channels, multiple of 16 */
    int32_t expand;    /* expansion of the inverted residual blocks, 1..16 */
    int32_t n_blocks;  /* inverted residual blocks, 0..16 */
} me_prnet_cfg;        /* widths: c_feat + c_enc + c_hid, expand*c_hid + c_hid <= 1024 */

typedef struct me_prnet_s* me_prnet;

typedef enum { ME_NHWC = 0, ME_NCHW = 1 } me_layout;

/* A device tensor of n images of HW pixels (layer calls): [n][HW][C]
 * (ME_NHWC) or [n][C][HW] (ME_NCHW); channels a multiple of 4. */
typedef struct {
    const void* data;
    int32_t channels;
    int32_t layout;    /* me_layout */
    int32_t dtype;     /* me_dtype */
} me_tensor;

/* Number of parameters of a configuration, or -1 if it is invalid. */
int64_t me_prnet_num_params(const me_prnet_cfg* cfg);

/* Create a network on the context's device (parameters unset: ME_E_STATE for
 * forward/train until me_prnet_set_params).  The network owns its parameters,
 * AdamW moments, packed operands and an activation workspace grown to the
 * largest call (growth synchronises the device). */
me_status me_prnet_create(me_ctx ctx, const me_prnet_cfg* cfg, me_prnet* out);
me_status me_prnet_destroy(me_prnet net);

/* Parameters from / to HOST memory (synchronous).  Setting them clears the
 * AdamW moments and step count. */
me_status me_prnet_set_params(me_prnet net, const float* params, int64_t count);
me_status me_prnet_get_params(me_prnet net, float* params, int64_t count);

/*
 * me_prnet_forward -- corrected features of n frames (paper Sec. 3.3):
 * cur = the first current mosaic (device), frame k at cur->data +
 * k * frame_stride elements; z_pred, z_out device [n][c_feat][Hf][Wf] in
 * `dtype` (ME_F32 or ME_BF16; z_out may not alias z_pred).  Asynchronous on
 * `stream`.  Calls on one network share its workspace: order them.
 */
me_status me_prnet_forward(me_prnet net, const me_frame* cur, int32_t n, int64_t frame_stride, const void* z_pred,
                           void* z_out, int32_t dtype, void* stream);

/*
 * me_prnet_forward_acts -- me_prnet_forward that also copies out the stage
 * outputs of the inference pass (paper Sec. 3.3: encoder, projection,
 * inverted residual blocks), so that its fused kernels can be checked stage
 * by stage: enc = device [n][Hf][Wf][c_enc] bfloat16 (the encoder output),
 * hid = device [n_blocks + 1][n][Hf][Wf][c_hid] bfloat16 (the projection
 * output, then each block's output).  Either may be NULL; the other
 * arguments, errors and ordering are those of me_prnet_forward.
 */
me_status me_prnet_forward_acts(me_prnet net, const me_frame* cur, int32_t n, int64_t frame_stride,
                                const void* z_pred, void* z_out, int32_t dtype, uint16_t* enc, uint16_t* hid,
                                void* stream);

/*
 * me_prnet_train_step -- forward, weighted BerHu loss against z_target, backward
 * (paper Sec. 3.3) and, when update != 0, one AdamW step (beta 0.9, 0.999,
 * eps 1e-8, weight decay 0.01, decoupled; learning rate lr).  z_pred, z_target:
 * device float32 [n][c_feat][Hf][Wf]; loss: device float (written); grads:
 * device float [num_params] or NULL (receives the gradient).  No gradient
 * flows into z_pred.  Asynchronous on `stream`; results are bit-reproducible.
 */
me_status me_prnet_train_step(me_prnet net, const me_frame* cur, int32_t n, int64_t frame_stride, const float* z_pred,
                              const float* z_target, float tau, float lr, int32_t update, float* grads, float* loss,
                              void* stream);

/* Single layers (device pointers; scratch in the context, so calls that share a
 * context must be ordered).  Depthwise 3x3, zero padding 1, stride 1 or 2:
 * x bfloat16 [n][H][W][C], w float32 [C][9], b float32 [C], y bfloat16
 * [n][ceil(H/s)][ceil(W/s)][C], ReLU6 when relu6 != 0. */
me_status me_prnet_dw_forward(me_ctx ctx, const uint16_t* x, const float* w, const float* b, int32_t n, int32_t H,
                              int32_t W, int32_t C, int32_t stride, int32_t relu6, uint16_t* y, void* stream);

/* Gradients of me_prnet_dw_forward given dy (bfloat16, output shape): dx
 * (bfloat16 [n][H][W][C], or NULL) times the ReLU6 derivative of `mask` (the
 * stored input activation, read where 0 < mask < 6; NULL = none), and grads
 * (float32 [C*9 + C]: weights then bias, or NULL). */
me_status me_prnet_dw_backward(me_ctx ctx, const uint16_t* x, const float* w, const uint16_t* dy, const uint16_t* mask,
                               int32_t n, int32_t H, int32_t W, int32_t C, int32_t stride, uint16_t* dx, float* grads,
                               void* stream);

/* 1x1 convolution over n*HW pixels: input channels = x then x2 (x2 NULL or
 * x2->data NULL for none); w float32 [cout][cin]; b [cout] or NULL; then
 * ReLU6 (relu6 != 0), + add (NULL for none), times the ReLU6 derivative of
 * mask (bfloat16 [n*HW][cout], NULL for none); written to out (cout channels,
 * any layout and dtype). */
me_status me_prnet_pw_forward(me_ctx ctx, const me_tensor* x, const me_tensor* x2, int32_t n, int32_t HW,
                              const float* w, const float* b, int32_t cout, int32_t relu6, const me_tensor* add,
                              const uint16_t* mask, const me_tensor* out, void* stream);

/* Gradients of a 1x1 convolution given dy (cout channels): grads (float32
 * [cout*cin + cout], weights then bias, or NULL) and dx (bfloat16 [n*HW]
 * [dx_count], or NULL) = the gradient of input channels dx_c0 .. dx_c0 +
 * dx_count - 1, + add (bfloat16, same shape, or NULL), times the ReLU6
 * derivative of mask (same shape, or NULL). */
me_status me_prnet_pw_backward(me_ctx ctx, const me_tensor* x, const me_tensor* x2, const me_tensor* dy, int32_t n,
                               int32_t HW, const float* w, int32_t cout, int32_t dx_c0, int32_t dx_count,
                               const uint16_t* add, const uint16_t* mask, uint16_t* dx, float* grads, void* stream);

/* The weighted BerHu loss alone: r, z_pred, z_target float32 [n][C][Hf][Wf];
 * dr (bfloat16, same shape) = dloss/dr; loss: device float. */
me_status me_prnet_loss(me_ctx ctx, const float* r, const float* z_pred, const float* z_target, int32_t n, int32_t C,
                        int32_t Hf, int32_t Wf, float tau, uint16_t* dr, float* loss, void* stream);

/*
 * me_sync -- wait until the work enqueued on `stream` (NULL = the null
 * stream) has finished.  Faults and launch failures of that asynchronous work
 * surface here: ME_E_HIP with the runtime's message in me_last_error().
 */
me_status me_sync(void* stream);

/*
 * Training-set statistics of the learned-proposal mode, computed on the GPU
 * from full-search SAD maps (device int32 [n][bh][bw] of n pairs of
 * frame_h x frame_w Bayer samples with blocks of `block` packed pixels).
 * The per-sample SAD of a block is q = sad / n_b in float32 (n_b = 4 h w, the
 * block's sample count).
 *
 * me_sad_median: *median (device float) = the lower median of q over all
 * n x bh x bw blocks (the element of rank floor((N-1)/2) in ascending order):
 * the M of the SAD fallback test (me_refine).  Scratch in the context.
 * me_fallback_weight: weight (device float32 [n][bh][bw]) = 1 where
 * sad <= floor(sad_ratio * median_per_sample * n_b) (product in double, left
 * to right: the SAD fallback threshold), else 0 -- blocks whose full-search
 * match is worse than any accepted proposal could be, left out of the vector
 * term of me_cnn_train_step.
 * Both asynchronous on `stream`; ME_E_INVAL on bad sizes.
 */
me_status me_sad_median(me_ctx ctx, const int32_t* sad, int32_t n, int32_t block, int32_t frame_h, int32_t frame_w,
                        float* median, void* stream);
me_status me_fallback_weight(const int32_t* sad, int32_t n, int32_t block, int32_t frame_h, int32_t frame_w,
                             float sad_ratio, float median_per_sample, float* weight, void* stream);

/* Human-readable name of a status code (static string). */
const char* me_status_string(me_status s);

/* Message describing the calling thread's last failed call (static per-thread
 * buffer, valid until the thread's next failing call). */
const char* me_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ME_H */
