// Library context and shared host-side helpers of the C ABI (not public).
#pragma once

#include <stdint.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/me.h"
#include "internal.h"

namespace me {

me_status fail(me_status s, const char* fmt, ...);
me_status hip_fail(hipError_t e, const char* what);
me_status check_frame(const me_frame* f, const char* name);
me_status check_pair(const me_frame* ref, const me_frame* cur);
bool block_ok(int B);
SearchArgs make_args(const me_frame* ref, const me_frame* cur, int B, int R, int limit, const int16_t* pred,
                     int16_t* mv, int32_t* sad);

// Proposal-network state: float32 master parameters, AdamW moments, the
// bfloat16 operand packings, and activation/gradient buffers sized for the
// largest batch seen so far.
// One queue launch of a batch plan: block size, tile shape, LDS bytes, its
// rows [first, first + n_jobs) of the queue table, item count and counter.
struct QueueLaunch {
    int block;
    TileCfg tile;
    size_t lds_bytes;
    int32_t first, n_jobs, n_items, counter;
};
constexpr int kQueueCounters = 8;
constexpr size_t kLdsQueue = 80 * 1024;      // two 8-wave workgroups per CU
constexpr size_t kLdsQueueMax = 158 * 1024;

struct CnnState {
    bool loaded = false;
    float* params = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* grads = nullptr;
    uint16_t* wf = nullptr;
    uint16_t* wb = nullptr;
    int64_t step = 0;
    int cap_n = 0, cap_hq = 0, cap_wq = 0;
    uint16_t* a0 = nullptr;   // pooled input of the proposal mode (one pair)
    uint16_t* a1 = nullptr;
    uint16_t* a2 = nullptr;
    uint16_t* a3 = nullptr;
    float* out = nullptr;
    uint16_t* dz4 = nullptr;
    uint16_t* d3 = nullptr;
    uint16_t* d2 = nullptr;
    uint16_t* d1 = nullptr;
    float* bl = nullptr;
    float* partial = nullptr;
    size_t partial_cap = 0;   // floats
    void release();
};

}  // namespace me

struct me_ctx_s {
    int device = 0;
    std::mutex mu;
    // launch shapes picked by the tuner, keyed by (B, R, Hp, Wp)
    std::map<std::tuple<int, int, int, int>, me::TileCfg> tuned;
    // proposal-mode scratch, grown on demand: decoded proposals, fallback
    // flags, the compacted fallback list and its device count
    int16_t* pred = nullptr;
    uint8_t* fb = nullptr;
    int32_t* list = nullptr;
    int32_t* count = nullptr;
    size_t cap_blocks = 0;
    // SAD per sample of the full-search best match, median over training data
    float median_per_sample = 0.0f;
    me::CnnState cnn;
    // batch submission: device table of per-pair pointers (grouped by shape),
    // its pinned host staging guarded by an event, and the captured graph of
    // the per-shape launches; a submission whose job shapes repeat the
    // previous one's (same order) replays the graph and only restages the
    // pointers
    me::JobPtrs* ptrs_dev = nullptr;
    me::JobPtrs* ptrs_host = nullptr;
    size_t cap_ptrs = 0;
    hipEvent_t staged = nullptr;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    std::vector<int64_t> batch_shapes;
    std::vector<int32_t> batch_slot;     // job k -> its row in the pointer table
    // queue launches of the batch plan: per-job geometry in launch order (the
    // job index of each row; pointers filled at each submission), the device
    // table and its pinned staging, the launches, and their ticket counters
    // (zero between launches)
    std::vector<me::QueueJob> qplan;
    std::vector<int32_t> qrow_job;
    std::vector<me::QueueLaunch> qlaunch;
    me::QueueJob* qjobs_dev = nullptr;
    me::QueueJob* qjobs_host = nullptr;
    size_t cap_q = 0;
    int32_t* qcount = nullptr;
    // pyramid search: vectors of the intermediate stages (ping-pong) and SADs
    int16_t* pyr_mv[2] = {nullptr, nullptr};
    int32_t* pyr_sad = nullptr;
    size_t pyr_cap = 0;
    // scratch of the single-layer network calls (packed weights, partials)
    void* prn_scratch = nullptr;
    size_t prn_scratch_cap = 0;
    // median selection: 256 counters and the (prefix, rank) state
    uint32_t* stat = nullptr;
    // autotune scratch outputs
    int16_t* tune_mv = nullptr;
    int32_t* tune_sad = nullptr;
    size_t tune_cap = 0;

    ~me_ctx_s();
};

namespace me {
me_status ensure_scratch(me_ctx ctx, size_t nblk);
TileCfg tiles_for(me_ctx ctx, int B, int R, int Hp, int Wp);
// Device scratch of the refine + fallback step: decoded proposals (int16
// [nblk][2], used for refine radii above 4), fallback flags (uint8 [nblk],
// used when the caller passes none), the compacted fallback list (int32
// [nblk]) and its count.
struct RefineScratch {
    int16_t* pred;
    uint8_t* fb;
    int32_t* list;
    int32_t* count;
};
// Refine + fallback given the median m and the scratch; no allocation.
me_status refine_run(const me_frame* ref, const me_frame* cur, const me_params& p, float m, const float* net_out,
                     int16_t* mv, int32_t* sad, uint8_t* fallback, const RefineScratch& w, hipStream_t st);
me_status check_refine_params(const me_params& p);
// Refine + fallback on a network output already in device memory.
me_status refine_impl(me_ctx ctx, const me_frame* ref, const me_frame* cur, const me_params& p, const float* net_out,
                      int16_t* mv, int32_t* sad, uint8_t* fallback, hipStream_t st);
// Resolve, with `device` made current for the call, the device address of
// the fixed scratch array of me_refine_noalloc (once per device).
me_status noalloc_resolve(int device);
// Pool + forward of one pair into ctx->cnn.out (proposal mode).
me_status cnn_propose(me_ctx ctx, const me_frame* ref, const me_frame* cur, hipStream_t st);
}  // namespace me
