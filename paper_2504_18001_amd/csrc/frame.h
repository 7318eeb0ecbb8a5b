// Device-side state of one frame and of the brick cache, and the host-side
// launch functions of the render and cache kernels.
#pragma once

#include <stddef.h>

#include "common.h"
#include "decision.h"

namespace cinr {

constexpr int kMaxIters = 8192;
constexpr int kClaimStride = 64;  // words between work-unit counters (separate cache lines)

enum : int32_t { S_HIT = 0, S_FALLBACK = 1, S_MISS = 2, S_SKIP = 3 };

enum StatIdx : int { ST_RAYS = 0, ST_SAMPLES, ST_HITS, ST_FALLBACKS, ST_MISSES, ST_SKIPPED, ST_REQUESTED, ST_SELECTED,
                     ST_EVICTED, ST_ITERS, ST_COUNT };

// Per wavefront iteration: rays live at its start, rays with a deferred
// wavefront step, true-miss records.
struct IterCtr {
    uint32_t live, pending, misses, pad;
};

// Cache-manager counters (device).
struct CacheCtr {
    uint32_t n_touched;   // bricks requested in the current frame
    uint32_t n_sel;       // bricks selected / to insert
    uint32_t n_free;      // free slots before the insertion
    uint32_t need_evict;  // slots to take from the LRU order
    uint32_t n_used;      // slots in use (free slots are [n_used, pool))
    uint32_t n_misslog;
    uint32_t n_evlog;
    uint32_t error;
    int32_t frame;        // frame whose requests are ranked; insertions are stamped frame + 1
    uint32_t select_done; // workgroups of the fused selection launch that have finished
    uint32_t n_views;     // views of the current frame (their statistics targets are in CacheDev::views)
    // the binary16 class of a mixed pool (slots [split, pool_bricks)); the
    // fields above then count the binary32 class, except n_sel (all bricks)
    uint32_t n_sel1, n_free1, need_evict1, n_used1;
    // two-level page table: free blocks on the stack, insertions left
    // unmapped for want of a block (never with the block pool's default size)
    uint32_t v_free, v_fail;
};

// Storage of the pool's brick values: one binary32 or one binary16 class of
// slots, or LoD-dependent mixed precision: binary32 slots [0, split) and
// binary16 slots [split, pool_bricks), each LoD stored in one class.
enum : int32_t { POOL_F32 = 0, POOL_F16 = 1, POOL_MIXED = 2 };

// Where a view's frame statistics go: written into the cache's table by the
// view's k_frame_begin, read at the end of the frame's selection.
struct ViewEnd {
    unsigned long long* stats;
    const IterCtr* ctr;
    int32_t max_iters, pad;
};
constexpr int kMaxFrameViews = 64;

struct MissLogRec {
    int32_t pix, k;
    float x, y, z;
};

struct CacheDev {
    int32_t* pt;
    int64_t* rank;
    uint32_t* req;
    uint32_t* last_req;   // nullable
    int32_t* touched;
    uint64_t* cand;
    int32_t* owner;
    int32_t* last_used;
    void* pool;           // binary32 slots [0, split), or every slot of a binary16 pool
    void* pool16;         // mixed pool: binary16 slot s at (s - split) * B^3
    int32_t* ins_keys;    // [ins_cap]
    int32_t* ins_slots;   // [ins_cap]
    int32_t* ins_reqs;    // [ins_cap][4]
    int32_t* ins_vols;    // [ins_cap] volume of each inserted brick
    uint64_t* topk[2];    // ping-pong buffers of the selection passes
    uint64_t* sel;        // final selection (sorted scores)
    uint64_t* vic;        // final victim list (sorted scores)
    MissLogRec* misslog;
    int32_t misslog_cap;
    int32_t* evlog;
    int32_t evlog_cap;
    CacheCtr* ctr;
    ViewEnd* views;       // [kMaxFrameViews]
    int32_t pool_bricks, max_requests, rank_window, ranking, ins_cap;
    int32_t pool_kind;    // POOL_F32, POOL_F16 or POOL_MIXED
    int32_t split;        // first slot of the binary16 class (pool_bricks unless mixed)
    uint32_t f16_lods;    // mixed: bit L set stores LoD L in the binary16 class
    uint64_t* vic1;       // victim list of the binary16 class (sorted scores)
    int32_t* ins_old;     // [ins_cap] key evicted by each insertion (-1: none)
    // two-level page table (vdir non-null; pt is then null): directory
    // [n_vols * dir_per_vol] of block ids (-1: no block), the block pool
    // [vcap][kVptEntries] of slots (-1: unmapped), the mapped entries of
    // each block, and the stack of free block ids (vfree[0, ctr->v_free))
    int32_t* vdir;
    int32_t* vblk;
    int32_t* vcnt;
    int32_t* vfree;
    int32_t vcap;
};

// Values of a view that change from one frame to the next while its launch
// sequence stays the same: the camera, the frame index, and the seed and floor
// of the stochastic LoD.  The kernels read them from device memory, where
// k_frame_begin copies them from a host block, so that the launches of a frame
// can be captured once and replayed.
struct FrameVar {
    CamDev cam;
    int32_t frame;
    uint32_t frame_seed;
    int32_t lod_floor;
    int32_t preload;  // a pre-load frame (Sec. 4.3.4): early ray termination suspended
    int32_t pad[9];
};
static_assert(sizeof(FrameVar) == 128, "FrameVar is copied as 32 words");

// Path tracing: the state of a pixel's paths between wavefront iterations
// (a pixel waits for the inference of its true misses), 128 bytes.
enum : uint32_t { PT_PRIMARY = 0, PT_SCATTER = 1, PT_SHADOW = 2 };
constexpr int kPtGather = 8;         // tentative collisions looked up from a true miss on, at most
constexpr uint32_t kPtMaxEvents = 8000;  // Philox events per pixel and frame
constexpr int kPtValsWord = 24;      // word offset of `vals` (inference writes there)
struct PtState {
    float o[3], d[3];      // current segment: origin and direction
    float t, te;           // t before the next event; end of the segment
    float beta[3];         // throughput of the path in progress
    float lp[3];           // radiance of the path in progress
    float sum[3];          // radiance of the completed paths
    uint32_t n;            // next event
    uint32_t path;         // index of the path in progress
    uint32_t done, hits;   // completed paths, and those whose primary ray collided
    uint32_t kind;         // PT_* | bounce << 2 | (primary collision) << 31
    uint32_t nc;           // values gathered from event n on
    uint32_t pad;
    float vals[kPtGather]; // their values (-1: skipped sample)
};
static_assert(sizeof(PtState) == 128 && offsetof(PtState, vals) == 4 * kPtValsWord, "PtState layout");

struct PtDev {
    int32_t on;            // the frame runs the path tracer
    float inv_sigma;       // 1 / pt_density (binary32)
    float ldir[3], light[3], ambient[3];
    int32_t bounces, spp, gather;
    uint32_t seed;
    PtState* st;           // [W*H]
};

struct FrameDev {
    int32_t W, H;  // image size (fixed for a view; the camera itself is in *var)
    FrameVar* var;            // device copy of the frame's values
    const FrameVar* var_src;  // host block (pinned) read by k_frame_begin; null: `var` is already stored
    int32_t dims[3];
    float vm1[3];
    float step, lod_scale, ert;
    int32_t ert_on;
    int32_t* ert_rec;     // nullable: per pixel, the grid index just past the sample whose
                          // compositing ended the ray early, -1 if it did not end early
    int32_t S;
    int32_t max_iters;    // bound on the wavefront iterations
    int32_t view_index, n_views;  // this view's place in the frame's views
    ViewEnd* view_table;  // nullable: the cache's table of the views' statistics targets
    int32_t mode;
    int32_t xcd_bands;  // image bands per XCD in the march kernel's work split
    int32_t claim_rev;  // 1: work units are claimed from the last one down
    int32_t pipe;       // samples fetched ahead per ray in the march kernel
    int32_t waves;      // waves per SIMD of the march kernel's register budget (3 or 4)
    int32_t mc_N;
    FastDiv div_mc;  // division by mc_N
    int32_t M[3];
    uint64_t* flags;     // nullable: one bit per macro-cell, set when the cell is visible
    int32_t flag_words;  // 64-bit words of `flags`
    // adaptive sampling rate: E > 0, then per macro-cell a code (0xFF
    // transparent, else the step exponent e <= E); 0: fixed step
    int32_t adapt;
    int32_t n_cells;
    uint8_t* cell_code;  // [n_cells]
    uint8_t* vexp;       // [W*H*S] step exponent of each gathered sample
    PtDev path;          // path tracing (path.on), else ray marching
    float lod_ctx;       // context-aware LoD weight (0: off)
    // Single-view frames: the first march's last workgroup writes the pending
    // count to *gather_host (pinned) and sets *gather_gate, in place of a
    // separate gather launch (null otherwise); exit_ticket counts its
    // finished workgroups (cleared by k_frame_begin).
    uint32_t* gather_host;
    uint32_t* gather_gate;
    uint32_t* exit_ticket;
    const float* minmax; // the volume's macro-cells [n_cells][2] (context-aware LoD)
    uint32_t* claim;     // [2][8] work-unit counters of the march kernel (one set per iteration
                         // parity), kClaimStride words apart
    CacheGeom geo;
    // cache (null in the uncached mode); pt and request keys are those of this
    // frame's volume: global key = key_base + key
    int32_t key_base;
    const int32_t* pt;
    // two-level page table instead of pt (vdir: this volume's directory)
    const int32_t* vdir;
    const int32_t* vblk;
    int32_t* last_used;
    uint32_t* req;
    int32_t* touched;
    uint32_t* n_touched;
    const void* pool;
    const void* pool16;  // binary16 class of a mixed pool
    int32_t pool_kind;   // POOL_F32, POOL_F16 or POOL_MIXED
    int32_t split;       // first binary16 slot of a mixed pool
    int32_t pool_bricks;
    MissLogRec* misslog;
    uint32_t* n_misslog;
    int32_t misslog_cap;
    // shading and ray state
    const float* tf;
    float4* rgba;
    int32_t* k_next;
    int32_t* live0;
    int32_t* live1;
    int32_t* pend_pix;
    int32_t* pend_n;
    float* vals;
    float4* miss_rec;
    IterCtr* ctr;
    unsigned long long* stats;
};

// Plan of the tournament top-k selection (blocks per pass).
constexpr int kTopkChunk = 2048;
constexpr int kMaxTopkPasses = 16;
constexpr int kMaxRequests = 256;  // each pass keeps k of 2048: at least 8:1 reduction
struct TopkPlan {
    int n_pass;
    int blocks[kMaxTopkPasses];
    uint32_t count[kMaxTopkPasses];  // input elements per pass (capacity)
};

inline TopkPlan make_topk_plan(int64_t cap, int k) {
    TopkPlan p{};
    int64_t c = cap;
    for (;;) {
        const int64_t b = (c + kTopkChunk - 1) / kTopkChunk;
        p.count[p.n_pass] = (uint32_t)c;
        p.blocks[p.n_pass] = (int)(b < 1 ? 1 : b);
        ++p.n_pass;
        if (b <= 1 || p.n_pass == kMaxTopkPasses) break;
        c = b * k;
    }
    return p;
}

enum TopkMode : int32_t { TOPK_SCORES = 0, TOPK_LRU = 1, TOPK_RANK = 2 };

struct RankArgs {
    const int32_t* touched;
    uint32_t* req;
    uint32_t* last_req;  // nullable
    int64_t* rank;
    const int32_t* frame;  // the cache's frame index (CacheCtr::frame)
    int32_t window, ranking;
};

struct SelectArgs {
    int32_t* ins_keys;
    CacheCtr* ctr;  // null: no epilogue
    int32_t pool_bricks, lim;
};

// Work the final selection workgroup does after publishing the request list:
// the insertion (when no LRU pass comes between) and the views' frame
// statistics.
struct SelectTail {
    int32_t insert, stats;
    CacheDev c;
    CacheGeom g;
};

struct TopkArgs {
    const uint64_t* in;
    const uint32_t* count_dev;  // live elements of pass 0 (nullable)
    uint64_t cap0;              // capacity of pass 0
    int32_t pass;
    uint64_t* out;
    int32_t k;
    const uint32_t* gate;       // nullable: skip when *gate == 0
    const uint32_t* frame_gate; // nullable: skip when *frame_gate == 0 (frame end queued ahead)
    int32_t mode;               // TopkMode of pass 0
    const int32_t* lru_last_used;
    int32_t lru_base;           // TOPK_LRU: slots [lru_base, lru_base + count)
    RankArgs ra;
    SelectArgs sel;
    // fused launch of a selection of two or more passes: the workgroups of
    // pass 0, then the last of them to finish runs the later passes alone
    // (through out and out2) into final_out
    int32_t fused;
    uint32_t* done;         // count of finished workgroups (reset by the last)
    uint64_t* final_out;
    uint64_t* out2;
    SelectTail tail;
    // passes of an unfused selection (the epilogue `sel` runs after the last);
    // when pass 0's live count fits one workgroup, that workgroup finishes the
    // selection and the later passes return at once
    int32_t last_pass;
};

// render.cpp launchers
// Macro-cell flags are staged in LDS by the march kernel up to this many words
// (131072 cells); larger grids are read from global memory.
constexpr int kMaxLdsFlagWords = 2048;
// ... and the adaptive sampler's one-byte cell codes up to this many cells.
constexpr int kMaxLdsCells = 32768;

hipError_t launch_frame_begin(const FrameDev& f, int32_t n_iter_ctr, const float* minmax, int64_t n_cells,
                              CacheCtr* cctr, hipStream_t s);
hipError_t launch_march(const FrameDev& f, int it, int64_t max_rays, hipStream_t s);
hipError_t launch_shade(const FrameDev& f, int it, int64_t cap_rays, hipStream_t s);
hipError_t launch_pt_free_flight(const uint32_t* words, int64_t n, float* out, hipStream_t s);
hipError_t launch_store_var(const FrameVar& v, FrameVar* dst, hipStream_t s);
// `gate` (nullable) on the frame-end launches: they do nothing unless *gate is
// non-zero, which k_pending_gather sets when no view has a ray pending after
// its iteration `it` (the first march, or the last iteration queued without
// a host round trip).  The end of a frame can so be queued before the host
// has read the pending counts.
hipError_t launch_frame_end(const FrameDev& f, int max_iters, CacheCtr* cctr, bool reset, const uint32_t* gate,
                            hipStream_t s);
hipError_t launch_pending_gather(const FrameDev* const* fs, int n, int it, uint32_t* host_out, uint32_t* gate,
                                 hipStream_t s);

// cache launchers
hipError_t launch_cache_init(const CacheDev& c, int64_t n_keys, int64_t n_dir, hipStream_t s);
// Two-level page table: the mapping changes of the last insertion batch.
hipError_t launch_vpt_update(const CacheDev& c, const CacheGeom& g, const uint32_t* gate, hipStream_t s);
// fuse_done (nullable): count of finished workgroups for a single fused
// launch of a two-pass plan (pass 0, then pass 1 in its last workgroup).
hipError_t launch_topk(const TopkArgs& base, const TopkPlan& plan, uint64_t* buf0, uint64_t* buf1, uint64_t* final_out,
                       const SelectArgs* epilogue, uint32_t* fuse_done, hipStream_t s);
hipError_t launch_prefill_setup(const CacheDev& c, const CacheGeom& g, const int32_t* keys, int32_t n, int32_t stamp,
                                hipStream_t s);
hipError_t launch_insert(const CacheDev& c, const CacheGeom& g, int32_t cap, const uint32_t* gate, hipStream_t s);
hipError_t launch_clear_last_req(const CacheDev& c, int64_t n_keys, hipStream_t s);

// inr.hip launchers
bool inr_shape_supported(const InrDev& m);
hipError_t inr_infer_points(const InrDev& m, const float* pos, int64_t n, float* out, int prec, hipStream_t s);
// gate: nullable, as for the frame-end launches (no brick is decoded unless *gate != 0)
hipError_t inr_decode_bricks(const InrDev& m, const CacheGeom& g, const int32_t* reqs, const uint32_t* n_dev,
                             const uint32_t* gate, int32_t n_cap, const int32_t* slots, const BrickOut& out,
                             int prec, hipStream_t s, DecodeShape shape = DecodeShape{});
hipError_t inr_macrocells(const InrDev& m, int32_t N, float* minmax, int prec, hipStream_t s);
hipError_t inr_infer_misses(const InrDev& m, const float4* rec, const uint32_t* n_dev, int64_t cap, float* vals,
                            int prec, hipStream_t s);
// bricks of several volumes of one shape (d_vols: device array of their
// descriptors, `shape` any of them on the host)
hipError_t inr_decode_bricks_multi(const InrDev* d_vols, const InrDev& shape, const CacheGeom& g, const int32_t* reqs,
                                   const int32_t* vols, const uint32_t* n_dev, const uint32_t* gate, int32_t n_cap,
                                   const int32_t* slots, const BrickOut& out, int prec, hipStream_t s, DecodeShape ds = DecodeShape{});

// train.hip launchers
bool train_shape_supported(const InrDev& m);
int32_t train_n_weights(const InrDev& m);
hipError_t train_gradients(const InrDev& m, int prec, const float* u, const float* target, int64_t n, float scale,
                           float* g_table, float* g_weights, float* loss, float* partial, int64_t max_waves,
                           hipStream_t s);
hipError_t train_points(uint64_t seed, int64_t step, int64_t n, const float* grid, const int32_t dims[3], float* u,
                        float* target, hipStream_t s);
hipError_t adam_update(float* p, float* m1, float* m2, float* g, int64_t n, float lr, float b1, float b2, float eps,
                       int64_t step, bool clear, hipStream_t s);
hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s);

}  // namespace cinr
