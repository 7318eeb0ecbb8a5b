/*
 * cinr.h -- C ABI of the MI355X (gfx950) cache-accelerated INR volume renderer.
 *
 * Implements the per-frame hot path of Zavorotny et al., "From Cluster to
 * Desktop: A Cache-Accelerated INR Framework for Interactive Visualization of
 * Tera-Scale Data": a scalar field defined only by a hash-grid INR (Section 3,
 * Figure 2) is ray marched (Section 5.1) through a multi-resolution brick cache
 * (Section 4.3): every sample looks up a per-LoD page table, falls back to
 * coarser LoDs, and interpolates trilinearly inside a brick of the pool; true
 * misses are inferred directly (Section 4.3.4, Algorithms 1 and 2); requested
 * bricks are ranked (Section 4.3.3) and decoded from the INR in batches
 * (Section 4.3.2) into the pool with LRU replacement (Figure 1, step (5)).
 *
 * Conventions shared by every entry point:
 *  - Plain C linkage; no C++ types, exceptions or STL cross this boundary.
 *  - Pointers prefixed d_ are device pointers (HIP device memory of the
 *    current device); other pointers are host pointers.
 *  - The caller owns every device buffer (parameters, pool, workspaces,
 *    images, statistics).  The library borrows them for the lifetime of the
 *    object or call and never frees them.  Library-owned memory is limited to
 *    host structs, one small pinned host buffer per volume, and the fixed
 *    device array of cinr_render_frame_noalloc.
 *  - `stream` is a hipStream_t (passed as void*); all work is enqueued on it.
 *    render_frame blocks the host until the first marching step of the frame
 *    has finished (it reads back the number of live rays to stop early);
 *    cinr_cache_dump synchronises the stream.  Nothing else synchronises.
 *  - Arguments are validated before any launch.  On failure the call returns
 *    a negative cinr_status and cinr_last_error() describes it (thread-local).
 *    Faults inside kernels surface at the next synchronising call.
 *  - Objects are not thread-safe; use one cache per stream.
 *  - Volume coordinates are LoD-0 voxel units; the volume box is
 *    [0, V-1]^3 (lattice points at integer coordinates).
 */
#ifndef CINR_H
#define CINR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CINR_OK = 0,
    CINR_INVALID_ARG = -1,
    CINR_OUT_OF_MEMORY = -2, /* a caller-provided buffer or workspace is too small */
    CINR_HIP_ERROR = -3,     /* the message holds the HIP error string */
    CINR_UNSUPPORTED = -4,   /* architecture, dtype or device not supported */
    CINR_BAD_STATE = -5
} cinr_status;

/* Arithmetic of the MLP layers (hash-grid interpolation, compositing and the
 * brick pool stay FP32; the output layer is FP32).  Reduced precisions run on
 * MFMA with FP32 accumulation.  CINR_BF16X3 splits every operand into two
 * BF16 terms (x = hi + lo) and accumulates hi*hi + hi*lo + lo*hi: BF16 MFMA
 * arithmetic with close to FP32 accuracy. */
typedef enum { CINR_F32 = 0, CINR_BF16 = 1, CINR_F16 = 2, CINR_BF16X3 = 3 } cinr_dtype;

typedef enum {
    CINR_CACHED = 0,          /* sampler of Algorithm 2 behind the brick cache */
    CINR_UNCACHED_DIRECT = 1, /* every sample inferred from the INR (the uncached baseline) */
    CINR_UNCACHED_LATTICE = 2 /* every sample the trilinear interpolation of the INR's values at its 8 LoD-0
                                 lattice points (cell clamped so that its upper corner exists): what a cache
                                 holding every LoD-0 brick renders, with no bricks.  Ray marching only;
                                 samples_per_iter >= 8, of which samples_per_iter / 8 samples per step */
} cinr_mode;

typedef enum {
    CINR_RANK_TIMESTAMP = 0, /* take this frame's requested bricks in key order (Section 4.3.3, default of Sarton et al.) */
    CINR_RANK_PRIORITY = 1   /* priority ranking of Section 4.3.3 */
} cinr_ranking;

typedef enum { CINR_PERSPECTIVE = 0, CINR_ORTHOGRAPHIC = 1 } cinr_projection;

#define CINR_MAX_LEVELS 32
#define CINR_MAX_LAYERS 8
#define CINR_MAX_LODS 16

/* A volume defined by a hash-grid INR (Section 3, Figure 2; value range of
 * Section 4.1; macro-cells of Section 5.2).
 *  dims          LoD-0 size (Vx, Vy, Vz), each >= 2.
 *  n_levels      grid levels m (<= 32); n_features entries per table slot
 *                (n, 1..4); log2_table: log2 of the per-level capacity T.
 *  level_res     per-level resolution N_l; level l stores
 *                T_l = min(T, (N_l+1)^3) entries; a level whose full grid fits
 *                is indexed densely (x + y(N+1) + z(N+1)^2), otherwise by the
 *                spatial hash (x*1 ^ y*2654435761 ^ z*805459861) mod T.
 *  n_layers, widths  MLP without biases: widths[0] = n_levels*n_features,
 *                widths[n_layers] = 1, ReLU between layers.
 *  value_scale, value_offset  value = clamp(scale*y + offset, 0, 1).
 *  d_table       f32 [sum_l T_l][n_features], level-major, under 4 GiB
 *                (CINR_INVALID_ARG otherwise).  Borrowed.
 *  d_weights     f32, layer k as [widths[k+1]][widths[k]] row-major,
 *                layers concatenated.  Borrowed.
 *  d_macrocells  optional f32 [ceil(Vz/N)][ceil(Vy/N)][ceil(Vx/N)][2] of
 *                (min, max) value per macro-cell of side macrocell_size N;
 *                NULL (and N = 0) disables empty-space skipping.  Borrowed.
 * The GPU path has kernels for 3 layers (two equal hidden layers of 32 or 64
 * neurons) with (n_levels, n_features) in {(8,2), (16,2), (16,4)}; other
 * shapes return CINR_UNSUPPORTED. */
typedef struct {
    int32_t dims[3];
    int32_t n_levels, n_features, log2_table;
    int32_t level_res[CINR_MAX_LEVELS];
    int32_t n_layers;
    int32_t widths[CINR_MAX_LAYERS + 1];
    float value_scale, value_offset;
    const float* d_table;
    const float* d_weights;
    const float* d_macrocells;
    int32_t macrocell_size;
} cinr_volume_desc;

/* Brick cache (Section 4.3.1).
 *  brick         stored samples per brick side B (2..64); neighbouring bricks
 *                share one sample per face, so a LoD-L brick spans
 *                (B-1)*2^L voxels (Section 4.3.2).
 *  n_lods        LoDs 0..n_lods-1 (<= 16).
 *  pool_bricks   brick slots in the pool (B^3 values each, of pool_dtype).
 *  max_requests  bricks requested and decoded per frame (maxNumRequests,
 *                at most 256).
 *  rank_window   ranks are clamped to timestamp + rank_window (1000).
 *  ranking       cinr_ranking.
 *  preload_period  pre-load of Section 4.3.4: the LoD floor starts at
 *                n_lods-1 and drops by one every preload_period frames
 *                (0 = off); the first preload_period frames (those forced
 *                to the coarsest LoD) march every ray to the end of the box,
 *                early ray termination suspended, so that the coarsest
 *                bricks behind opaque material are requested too.
 *  miss_log_capacity   true-miss records kept per frame for dumps (0 = off).
 *  evict_log_capacity  insertion/eviction records kept for dumps.
 *  keep_request_counts nonzero: keep each frame's per-brick request counts
 *                for CINR_DUMP_REQ_COUNT.
 *  pool_dtype    CINR_F32 (0) or CINR_F16: binary16 brick values (decoded
 *                values rounded to nearest, ties to even), half the pool
 *                memory; the sampler interpolates them in FP32 (a reduced-
 *                precision pool, the paper's future work, Sec. 7).
 *  f16_lods, pool_bricks_f16  LoD-dependent mixed precision (Sec. 7's
 *                future work: an encoding per LoD).  0 = one class of
 *                pool_dtype.  Otherwise bit L of f16_lods stores LoD L's
 *                bricks as binary16 (rounded as above) in the slots
 *                [pool_bricks - pool_bricks_f16, pool_bricks), and the other
 *                LoDs as binary32 in the slots below.  A brick takes a slot of
 *                its class only: the class's lowest free slot, else the
 *                class's least recently used slot (same order as the one-class
 *                pool).  Requires pool_dtype = CINR_F32, a non-empty proper
 *                subset of the LoDs, and max_requests <= the slots of each
 *                class.  A LoD whose error bound admits binary16 rounding
 *                (at most 2^-12 for the pool's values in [0, 1]) can take
 *                the binary16 class.
 *  virtual_page_table  0: one flat page table entry per brick key (4 bytes
 *                per brick of every LoD).  1: the virtualised page tables of
 *                Section 4.3.1, two levels: a directory entry per block of
 *                8^3 bricks of a LoD (4 bytes per 512 bricks) points to a
 *                block of 512 entries (2 KiB) taken from a block pool when
 *                one of its bricks is mapped and returned when the last one
 *                is unmapped.  The sampler reads the directory, then the
 *                block.  The mapping (brick -> slot), and so every frame's
 *                results, equal those of the flat table.
 *  pt_blocks     blocks of the block pool (virtual_page_table = 1); 0 takes
 *                min(directory entries, pool_bricks), which can never run
 *                out (each block in use holds a mapped brick).  Below that, a
 *                brick whose block cannot be had stays unmapped (counted in
 *                CINR_DUMP_PT_STATE) and frames may differ from the flat
 *                table's.
 */
typedef struct {
    int32_t brick, n_lods, pool_bricks, max_requests, rank_window;
    int32_t ranking;
    int32_t preload_period;
    int32_t miss_log_capacity;
    int32_t evict_log_capacity;
    int32_t keep_request_counts;
    int32_t pool_dtype;
    uint32_t f16_lods;
    int32_t pool_bricks_f16;
    int32_t virtual_page_table;
    int32_t pt_blocks;
} cinr_cache_desc;

/* Pinhole or orthographic camera.  Basis vectors are unit length; pixel
 * (i, j) (row j = 0 at the top) maps to screen offsets
 * sx = ((i+0.5)/W*2-1)*tan_half_x, sy = (1-(j+0.5)/H*2)*tan_half_y
 * (perspective), or to an origin offset ((i+0.5)/W-0.5)*ortho_w along right
 * and (0.5-(j+0.5)/H)*ortho_h along up (orthographic).  The LoD distance of
 * Algorithm 2 is measured from `eye`. */
typedef struct {
    int32_t projection, width, height;
    float eye[3], forward[3], right[3], up[3];
    float tan_half_x, tan_half_y, ortho_w, ortho_h;
} cinr_camera;

/* Per-frame parameters.
 *  step          sample spacing (LoD-0 voxels); opacity is corrected from a
 *                one-voxel reference: a' = 1 - (1-a)^step.
 *  lod_scale     LoD distance |p - eye| * lod_scale (Algorithm 2).
 *  ert_threshold early ray termination at accumulated opacity >= threshold;
 *                a value > 1 disables it.
 *  seed, frame_index  the stochastic-LoD seed of frame f is derived from
 *                (seed, f) (Section 5.3); frame_index is also the cache's
 *                timestamp and must increase by one per cached frame.
 *  samples_per_iter  samples gathered per wavefront step after a true miss.
 *  mode          cinr_mode.
 *  mlp_dtype     cinr_dtype of brick decoding and true-miss inference.
 *  pipe_depth    tuning: samples each ray decides and fetches ahead while
 *                marching (1, 2 or 4; 8 is accepted and runs as 4).
 *  xcd_bands     tuning: image bands per XCD in the sampler's work split
 *                (1 to 64).
 *  waves_per_simd tuning: the sampler's register budget, 3 waves per SIMD
 *                (168 registers, no spills) or 4 (128 registers); 0 takes
 *                the tuned value, or 3 when the launch is not tuned; frames
 *                of several views (cinr_render_views, frame graphs) take 4,
 *                since their views march concurrently.
 *                Results depend on none of them.  0 in pipe_depth or
 *                xcd_bands tunes the launch online, per volume and image
 *                size: frames of that size try pipe depths {1, 2} x bands
 *                {1, 4, 16} x waves {3, 4} x the two claim directions of the
 *                image tiles (first tile first, or last tile first) twice
 *                each (48 trials, the second round in reverse order), then
 *                the candidate with the
 *                lowest first-march time per sample is kept
 *                (cinr_tuned_launch reports the choice); each counted trial
 *                reads the frame's sample count back, with a synchronisation
 *                of the view's stream.  Frames under a pre-load LoD floor
 *                are not counted.  A
 *                frame whose first march leaves rays waiting on true misses
 *                is not counted (its march was cut short) until 96 such
 *                frames have passed.
 *  adapt_max_exp adaptive sampling rate (Section 5.2), with the volume's
 *                macro-cells: E > 0 lets a ray cross a macro-cell of maximum
 *                TF opacity mu in steps of 2^e sample spacings, e =
 *                min(E, floor(-log2 mu)), still on its grid ts + k*step
 *                (sample k is followed by sample k + 2^e), each sample's
 *                opacity corrected to its own step; a transparent cell is
 *                crossed in steps of 2^E with its samples skipped.  0 (or
 *                no macro-cells) is the fixed step; at most 14.  The march
 *                runs with pipe depth 1 in this mode. */
typedef struct {
    float step, lod_scale, ert_threshold;
    uint32_t seed;
    int32_t frame_index;
    int32_t samples_per_iter;
    int32_t mode;
    int32_t mlp_dtype;
    int32_t pipe_depth;
    int32_t xcd_bands;
    int32_t adapt_max_exp;
    int32_t waves_per_simd;   /* tuning (see above): 3, 4, or 0 */
    /* Path tracing (pipeline = CINR_PATH_TRACE): the second wavefront
     * pipeline of Section 5.1, Woodcock delta tracking through the same
     * sampler and cache.  The medium has extinction pt_density * TF opacity
     * per LoD-0 voxel (pt_density is the majorant), the TF colour as
     * scattering albedo and an isotropic phase function.  Each path tracks
     * the primary ray; at a real collision its throughput takes the albedo, a
     * shadow ray toward pt_light_dir (unit vector, used as given) is tracked
     * the same way and adds throughput * pt_light when it leaves the box
     * (pt_light carries the phase factor), then the path scatters in a
     * uniform direction (Marsaglia's method), up to pt_max_bounces
     * collisions; a scattered ray that leaves the box adds throughput *
     * pt_ambient.  A tentative collision is real when a uniform falls below
     * the TF opacity at the sampled value (binary32); free flights are
     * -ln(xi) / pt_density with xi = ((r >> 8) + 1) 2^-24, the logarithm in
     * binary64 rounded to binary32.  Random words: Philox-4x32-10, key
     * (pt_seed, frame_index), counter (pixel, event, 0, 0), events numbered
     * per pixel across its paths; a pixel draws at most 8000 events per frame
     * (a path cut by that budget is dropped).  The pixel's colour is the mean
     * radiance of its pt_spp paths, its opacity the fraction of those whose
     * primary ray collides.  From a true miss on, up to min(samples_per_iter,
     * 8) tentative collisions of the segment are looked up and inferred
     * together (the wavefront step of the ray marcher); this changes the
     * lookup counts, never a path.  step, ert_threshold and the tuning
     * fields are not used; adapt_max_exp must be 0.  The workspace is sized
     * by cinr_path_workspace_size. */
    int32_t pipeline;         /* cinr_pipeline */
    float pt_density;         /* > 0 */
    float pt_light_dir[3];
    float pt_light[3];
    float pt_ambient[3];
    int32_t pt_max_bounces;   /* >= 1 */
    int32_t pt_spp;           /* 1 .. 65535 */
    uint32_t pt_seed;
    /* Context-aware LoD (the direction of Section 7: use the macro-cells'
     * value ranges to pick finer LoDs where the data has structure): with
     * macro-cells, the LoD distance of a sample in a cell of values
     * [min, max] is (|p - eye| * lod_scale) * (1 - lod_context * (max - min)),
     * in binary32; 0 (or no macro-cells) is Algorithm 2's distance rule.
     * In [0, 1]. */
    float lod_context;
    /* Optional output (ray marching only, NULL otherwise): where each ray
     * of the frame ended early, so that a checker can replay the frame's
     * early terminations sample for sample (the performance mode, with
     * early ray termination on): int32 [height][width] device memory, borrowed for the
     * call (for frame graphs: for the graph's lifetime).  The frame writes
     * for every pixel the sample-grid index k + 1 of the sample k whose
     * compositing brought the accumulated opacity to ert_threshold (the
     * grid index the ray would have sampled next; with the adaptive rate,
     * k + 2^e), or -1 when the ray was not ended early (it left the box, did
     * not hit it, or early termination was off).  The frames of the
     * pre-load (frame_index < preload_period of the cache) march without
     * early termination, so they record -1 everywhere. */
    int32_t* ert_record;
} cinr_render_params;

typedef enum { CINR_RAY_MARCH = 0, CINR_PATH_TRACE = 1 } cinr_pipeline;

/* Frame counters written (not accumulated) by cinr_render_frame. */
typedef struct {
    uint64_t rays, samples, hits, fallbacks, misses, skipped;
    uint64_t requested, selected, evicted, iterations;
} cinr_frame_stats;

typedef enum {
    CINR_DUMP_PAGE_TABLE = 0,   /* int32 [n_keys]: slot or -1 */
    CINR_DUMP_SLOT_OWNER = 1,   /* int32 [pool_bricks]: key or -1 */
    CINR_DUMP_LAST_USED = 2,    /* int32 [pool_bricks]: last frame that read the slot, -1 never */
    CINR_DUMP_RANK = 3,         /* int64 [n_keys]: rank, -1 undefined */
    CINR_DUMP_REQ_COUNT = 4,    /* uint32 [n_keys]: requests of the last frame (keep_request_counts) */
    CINR_DUMP_REQUEST_LIST = 5, /* int32 [n]: keys selected at the end of the last frame, in order */
    CINR_DUMP_MISS_LIST = 6,    /* {int32 pixel, int32 k, float x, y, z} [n] of the last frame, sorted by (pixel, k);
                                   k is the sample index (ray marching) or the event index (path tracing, where a
                                   (pixel, k) pair can repeat: an event looked up ahead after a true miss is drawn
                                   again by the segment that follows a real collision) */
    CINR_DUMP_EVICTION_LOG = 7, /* {int32 stamp, slot, old_key, new_key} [n] since creation */
    CINR_DUMP_POOL = 8,         /* pool_dtype values [pool_bricks][B][B][B]: float, or binary16 bits; a mixed
                                   pool: float [split][B][B][B], then binary16 bits [pool_bricks - split][B][B][B] */
    CINR_DUMP_PT_DIRECTORY = 9, /* two-level page table: int32 [n_vols][directory entries]: block or -1 */
    CINR_DUMP_PT_BLOCKS = 10,   /* two-level page table: int32 [blocks][512]: slot or -1 */
    CINR_DUMP_PT_STATE = 11     /* two-level page table: int32 {blocks, free blocks, insertions left unmapped
                                   for want of a block, directory entries per volume} */
} cinr_dump_kind;

typedef struct cinr_volume_s* cinr_volume;
typedef struct cinr_cache_s* cinr_cache;

/* Validates the description and binds the borrowed parameter buffers.
 * Computes the per-level table layout on the host.  No device work. */
cinr_status cinr_create_volume_inr(const cinr_volume_desc* desc, cinr_volume* out);

/* A volume defined by an explicit voxel grid (the fallback source of the
 * learned part and the reference its INR is judged against): d_grid is f32
 * [Vz][Vy][Vx], x fastest, borrowed for the volume's lifetime.  The value at
 * voxel coordinate x is the trilinear interpolation of the samples at x
 * (clamped to [0, V-1]), then clamp(value_scale * v + value_offset, 0, 1).
 * Every volume operation accepts it (their mlp_dtype arguments are
 * ignored); training does not. */
typedef struct {
    int32_t dims[3];       /* >= 2 each */
    const float* d_grid;
    float value_scale, value_offset;
    const float* d_macrocells;  /* optional, as for INR volumes */
    int32_t macrocell_size;
} cinr_grid_desc;
cinr_status cinr_create_volume_grid(const cinr_grid_desc* desc, cinr_volume* out);
void cinr_destroy_volume(cinr_volume vol);

/* LoD lattice and bricks of Section 4.3.2: at LoD L the lattice step is 2^L,
 * K_L = ceil((V-1)/2^L) + 1 points per axis, nb_L = ceil((K_L-1)/(B-1))
 * bricks per axis; keys are numbered LoD by LoD, x fastest.
 * Writes nb [n_lods][3] and key_offset [n_lods+1] (host arrays, either may be
 * NULL); key_offset[n_lods] is the number of keys. */
cinr_status cinr_lod_geometry(cinr_volume vol, int32_t brick, int32_t n_lods, int32_t* nb, int64_t* key_offset);

/* Evaluates the INR (InferINR of Algorithm 1) at n positions d_pos
 * (f32 [n][3], voxel coordinates, clamped to the box) into d_out (f32 [n]). */
cinr_status cinr_infer_points(cinr_volume vol, const float* d_pos, int64_t n, float* d_out, int32_t mlp_dtype,
                              void* stream);

/* Brick decoding of Section 4.3.2 (the request handler's INR integration).
 * d_reqs int32 [n][4] = (lod, bx, by, bz); d_out f32 [n][B][B][B] in
 * (z, y, x) order; element (r, k, j, i) is the value at voxel coordinate
 * clamp((b*(B-1) + (i, j, k)) * 2^lod, 0, V-1).  Requests are checked on the
 * device: an out-of-range request yields a brick of NaNs. */
cinr_status cinr_decode_bricks(cinr_volume vol, const int32_t* d_reqs, int32_t n, int32_t brick, float* d_out,
                               int32_t mlp_dtype, void* stream);

/* Brick decoding with an explicit launch shape, for tuning and tests.
 * parts_per_brick = 0: one point per lane over the whole request list, every
 * corner read from the hash table (the layout of cinr_infer_points).
 * Otherwise (brick <= 16; a larger brick uses parts_per_brick = 0) a
 * workgroup takes one of P slabs of z-slices of a brick, where P is at least
 * parts_per_brick (1, 2, 4, 8 or 16; a divisor of `brick`) and is doubled on
 * the device, while it divides the brick and stays <= 16, until the launch's
 * request count gives every resident workgroup a slab (short request lists).  The lattice coordinates of a brick
 * are separable, so each hash-grid level's cells and weights are computed per
 * axis once per slab.  With stage_kib 32 or 64 (0: none), for each level the
 * box of grid corners that the slab's lattice points touch is also copied
 * into LDS once, smallest boxes first while they fit in stage_kib KiB and
 * cost fewer reads than the points' own corner reads, and the slab's points
 * interpolate those levels from LDS (Section 3's encoding over the regular
 * lattice of a brick, Section 4.3.2).  Every shape gives the same bits. */
cinr_status cinr_decode_bricks_shaped(cinr_volume vol, const int32_t* d_reqs, int32_t n, int32_t brick,
                                      float* d_out, int32_t mlp_dtype, int32_t parts_per_brick, int32_t stage_kib,
                                      void* stream);
/* The launch shape (as above) that cinr_decode_bricks and the caches of this
 * volume use for its brick decoding; the default is parts_per_brick = 0. */
cinr_status cinr_set_decode_shape(cinr_volume vol, int32_t parts_per_brick, int32_t stage_kib);
/* Autotuner of the decoding launch shape: decodes the n requests d_reqs
 * (for example a recent request list) into d_out (scratch of n * brick^3
 * floats) once per candidate shape to warm up and then `reps` times, timed
 * with HIP events on `stream` (which is synchronised), sets the fastest as
 * the volume's decode shape and returns its index in *chosen (nullable).
 * ms_out (host, nullable) receives the 16 candidates' milliseconds per
 * decode in this order of (parts_per_brick, stage_kib): (0, 0), then for
 * parts_per_brick 1, 2, 4, 8 and 16 in turn stage_kib 0, 32 and 64; -1 for a
 * shape `brick` does not admit.  Creates two events. */
cinr_status cinr_tune_decode(cinr_volume vol, const int32_t* d_reqs, int32_t n, int32_t brick, float* d_out,
                             int32_t mlp_dtype, int32_t reps, float* ms_out, int32_t* chosen, void* stream);

/* Macro-cell table of Section 5.2 built from the INR itself: for each cell of
 * side `cell`, min and max of the LoD-0 lattice values in its closed region
 * [cN, min((c+1)N, V-1)]^3, written to d_minmax (layout as d_macrocells). */
cinr_status cinr_build_macrocells(cinr_volume vol, int32_t cell, float* d_minmax, int32_t mlp_dtype, void* stream);

/* Size of the caller-provided cache workspace (page table, ranks, request
 * counts, slot owners and stamps, request and log buffers). */
cinr_status cinr_cache_workspace_size(cinr_volume vol, const cinr_cache_desc* desc, size_t* bytes);

/* Creates a cache over a caller-provided pool and workspace; initialises
 * the workspace on `stream` (all bricks unmapped, all slots free).  The pool
 * holds pool_bricks*B^3 values of pool_dtype, or for a mixed pool
 * (pool_bricks - pool_bricks_f16)*B^3 binary32 values followed by
 * pool_bricks_f16*B^3 binary16 values. */
cinr_status cinr_create_cache(cinr_volume vol, const cinr_cache_desc* desc, void* d_pool, size_t pool_bytes,
                              void* d_workspace, size_t ws_bytes, void* stream, cinr_cache* out);
void cinr_destroy_cache(cinr_cache cache);

/* Pre-loading: inserts the bricks d_keys [n] (distinct, unmapped keys) into
 * free slots, in order, as the request handler would at the start of a frame
 * stamped `stamp`: decoded, mapped and stamped.  Keys beyond the free slots
 * are not inserted (pre-loading never evicts).  n <= min(pool, n_keys). */
cinr_status cinr_cache_prefill(cinr_cache cache, const int32_t* d_keys, int32_t n, int32_t stamp, int32_t mlp_dtype,
                               void* stream);

/* Size of the per-call render workspace (ray lists, sample buffers, miss
 * records, counters, macro-cell flags) for a width x height image. */
cinr_status cinr_render_workspace_size(cinr_volume vol, int32_t width, int32_t height, int32_t samples_per_iter,
                                       size_t* bytes);

/* Size of the render workspace of the path tracer: the ray marcher's plus
 * 128 bytes of path state per pixel (width * height < 2^27). */
cinr_status cinr_path_workspace_size(cinr_volume vol, int32_t width, int32_t height, int32_t samples_per_iter,
                                     size_t* bytes);

/* The path tracer's free-flight lengths for n random words (device arrays):
 * d_out[i] = -ln(((d_words[i] >> 8) + 1) * 2^-24), computed in binary64 and
 * rounded to binary32, exactly as the renderer draws them. */
cinr_status cinr_pt_free_flight(const uint32_t* d_words, int64_t n, float* d_out, void* stream);

/* Renders one frame into d_rgba (f32 [H][W][4], straight colour and
 * opacity, no background).
 *  CACHED mode: `cache` must be non-NULL; the frame runs the sampler against
 *  the cache, then the end-of-frame cache manager (ranking, request list) and
 *  the request handler (slot choice, brick decoding, mapping), so that the
 *  next frame starts with the new bricks (latency of one frame).
 *  UNCACHED_DIRECT mode: `cache` is ignored; every sample is inferred.
 *  d_tf f32 [256][4] RGBA transfer function (Section 3), linearly
 *  interpolated at value*255.  d_stats (nullable) receives the counters. */
cinr_status cinr_render_frame(cinr_cache cache, cinr_volume vol, const cinr_camera* camera, const float* d_tf,
                              const cinr_render_params* params, float* d_rgba, cinr_frame_stats* d_stats,
                              void* d_workspace, size_t ws_bytes, void* stream);

/* Allocation-free variant of cinr_render_frame, for callers that cannot
 * allocate memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and cache state machine
 * as cinr_render_frame, without the render workspace: the frame's scratch
 * (ray lists, gathered samples, miss records, counters) lives in a fixed
 * device array of CINR_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device it runs on until the process ends.
 *  - No device or pinned-host memory is allocated, no HIP event or stream is
 *    created.  The pending-ray count is read back with a copy into host
 *    memory followed by a synchronisation of `stream`, so this call blocks
 *    until the frame has finished (cinr_render_frame waits only for the first
 *    marching step).
 *  - A launch shape left to the tuner (pipe_depth or xcd_bands 0) takes the
 *    shape already tuned for this image size, else the first candidate; no
 *    launch-shape trial runs.  Stage timing is not recorded.
 *  - Returns CINR_OUT_OF_MEMORY, before any launch, when the frame needs more
 *    than CINR_NOALLOC_SCRATCH_BYTES - 256 bytes of workspace (the size
 *    cinr_render_workspace_size or cinr_path_workspace_size reports; about
 *    21 * samples_per_iter + 40 bytes per pixel for ray marching).
 *  - Every call on one device shares that device's array and leaves its
 *    contents behind; each frame clears what it needs cleared.  Calls that
 *    overlap on one device (several host threads, or streams that run
 *    concurrently) race on the array and must not be issued. */
#define CINR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
cinr_status cinr_render_frame_noalloc(cinr_cache cache, cinr_volume vol, const cinr_camera* camera, const float* d_tf,
                                      const cinr_render_params* params, float* d_rgba, cinr_frame_stats* d_stats,
                                      void* stream);

/* Optional per-stage GPU timing of cinr_render_frame, for profiling.
 * While enabled, every stage launch of render_frame is bracketed by HIP
 * events on the caller's stream (no synchronisation is added);
 * cinr_collect_timing synchronises on the last event, writes the summed
 * milliseconds and the number of bracketed launches per stage
 * (arrays of CINR_STAGE_COUNT) and clears the record.  enable: 0 off,
 * 1 every stage, 2 the march stage only (two events per march launch, the
 * least overhead). */
typedef enum {
    CINR_STAGE_SETUP = 0,   /* frame initialisation, macro-cell flags, ray generation */
    CINR_STAGE_MARCH = 1,   /* sampler: cache lookups, compositing, miss gathering */
    CINR_STAGE_INFER = 2,   /* true-miss inference */
    CINR_STAGE_SHADE = 3,   /* compositing of gathered wavefront steps */
    CINR_STAGE_CM = 4,      /* ranking, request selection, slot choice, mapping */
    CINR_STAGE_DECODE = 5,  /* brick decoding into the pool */
    CINR_STAGE_COUNT = 6
} cinr_stage;
cinr_status cinr_set_timing(cinr_volume vol, int32_t enable);
cinr_status cinr_collect_timing(cinr_volume vol, double* ms, int64_t* launches);

/* A cache shared by several volumes (for instance several INRs seen by
 * several views): all volumes must have the same dimensions and the same
 * kind and shape (INRs with equal levels, features and widths, or grids).
 * Volume i owns the keys [i * K, (i + 1) * K), where K is the key count of
 * one volume (cinr_lod_geometry); page table, request counts, ranks and the
 * pool are shared, and the bricks selected in a frame are decoded in one
 * persistent launch whatever their volumes.  The volumes must outlive the
 * cache.  cinr_create_cache is the case of one volume. */
cinr_status cinr_cache_workspace_size_multi(const cinr_volume* vols, int32_t n_vols, const cinr_cache_desc* desc,
                                            size_t* bytes);
cinr_status cinr_create_cache_multi(const cinr_volume* vols, int32_t n_vols, const cinr_cache_desc* desc,
                                    void* d_pool, size_t pool_bytes, void* d_workspace, size_t ws_bytes,
                                    void* stream, cinr_cache* out);

/* One view of a multi-view frame. */
typedef struct {
    cinr_volume volume;          /* one of the cache's volumes */
    cinr_camera camera;
    const float* d_tf;           /* f32 [256][4] */
    cinr_render_params params;   /* CACHED; frame_index and mlp_dtype equal in all views */
    float* d_rgba;               /* f32 [H][W][4] */
    cinr_frame_stats* d_stats;   /* nullable; the request counters are the frame's */
    void* d_workspace;           /* this view's render workspace (cinr_render_workspace_size) */
    size_t workspace_bytes;
} cinr_view;

/* Renders one frame of several views through a shared cache: every view is
 * marched against the residency at the start of the frame, then one cache
 * manager pass ranks the requests of all views and the selected bricks are
 * decoded in one launch (the frame advances the cache by exactly one frame,
 * as cinr_render_frame does for one view).  The views' first iterations are
 * launched back to back and synchronised once. */
cinr_status cinr_render_views(cinr_cache cache, int32_t n_views, const cinr_view* views, void* stream);

/* Captured multi-view frames (hipGraph).  A frame graph is made for a fixed
 * set of views: volumes, image sizes and projections, TF, image, statistics
 * and workspace pointers, and every render parameter except frame_index.
 * Each cinr_frame_graph_render call renders one frame of those views with new
 * cameras and a new frame index, with the same results as cinr_render_views
 * (bit for bit), by replaying one captured graph per frame: the set-up and
 * first march of every view (on the cache's side streams, as in
 * cinr_render_views), K further wavefront iterations of every view (true-miss
 * inference, shading, march; K = 0 unless set by
 * cinr_frame_graph_set_device_iterations), the pending-ray counts of all
 * views after them written to pinned host memory, then ranking, request
 * selection, insertion, decoding and the frame ends, which the device skips
 * while any view has pending rays.  The queued iterations size their launches
 * for every pixel and read their ray counts on the device (an iteration with
 * no ray pending ends at once), so a frame that needs at most K + 1
 * iterations makes no host round trip before its end.  The host waits for the
 * pending counts; views that still have pending rays finish their wavefront
 * iterations with ordinary launches, followed by the frame end.  The camera, frame index and LoD seed are read
 * from device memory that the graph fills from a host block, so the graph
 * does not change from frame to frame; two graphs are kept, with and without
 * the LRU victim pass.  While a view's launch shape is being tuned
 * online (pipe_depth or xcd_bands 0), frames are rendered as by
 * cinr_render_views and nothing is captured.  Stage timing does not cover
 * graph frames.  The TF contents may change between frames (the macro-cell
 * visibility is recomputed by every frame).  The graph borrows the cache,
 * the volumes and every buffer of the views; destroy it first.  Calls on one
 * graph, or on graphs of one cache, must not overlap.
 * Errors: CINR_INVALID_ARG (as cinr_render_views; a camera whose size or
 * projection differs from the one the graph was made with), CINR_HIP_ERROR
 * (capture, instantiation or launch). */
typedef struct cinr_frame_graph_s* cinr_frame_graph;
cinr_status cinr_frame_graph_create(cinr_cache cache, int32_t n_views, const cinr_view* views, cinr_frame_graph* out);
/* cameras: [n_views], in the order of the views given at creation. */
cinr_status cinr_frame_graph_render(cinr_frame_graph graph, const cinr_camera* cameras, int32_t frame_index,
                                    void* stream);
/* Wavefront iterations after the first march that the graph queues on the
 * device (K above; 0 to 16, clamped to each view's iteration bound).  A new
 * value synchronises the device and drops the captured graphs, which are
 * captured again on their next use.  Errors: CINR_INVALID_ARG, CINR_HIP_ERROR. */
cinr_status cinr_frame_graph_set_device_iterations(cinr_frame_graph graph, int32_t iterations);
/* Frames rendered from the graphs, frames rendered eagerly (launch shape
 * still being tuned), and graph frames that needed further iterations. */
cinr_status cinr_frame_graph_counts(cinr_frame_graph graph, int64_t* graph_frames, int64_t* eager_frames,
                                    int64_t* tail_frames);
void cinr_frame_graph_destroy(cinr_frame_graph graph);

/* The sampler launch shape tuned online for a volume and image size (see
 * cinr_render_params), and the trial frames still to run (0 once tuned). */
cinr_status cinr_tuned_launch(cinr_volume vol, int32_t width, int32_t height, int32_t* pipe_depth,
                              int32_t* xcd_bands, int32_t* waves_per_simd, int32_t* trials_left);

/* Copies one piece of cache state to host memory.  If `bytes` is too small
 * (or host_dst is NULL) nothing is copied, *needed receives the size and
 * CINR_OUT_OF_MEMORY is returned.  Synchronises `stream`. */
cinr_status cinr_cache_dump(cinr_cache cache, int32_t kind, void* host_dst, size_t bytes, size_t* needed,
                            void* stream);

/* ------------------------------------------------------------------------
 * Training of the volume's INR (the learned part; Section 4.1 fits the INR
 * to the data).  Loss: mean over a batch of (y - target)^2, with y the raw
 * MLP output (no value normalisation) at points u in [0,1)^3.  Gradients flow
 * through the MLP and the hash-grid interpolation into every table entry and
 * weight; Adam (Kingma and Ba) updates all of them.  The trainer writes the
 * volume's parameter buffers (d_table, d_weights) in place: they must be
 * writable, and the volume's value_scale/value_offset should be 1/0.
 *
 * Points of step s: Philox-4x32-10 with counter (i, s) and key `seed`, 24 bits
 * per coordinate.  Target of a point: trilinear interpolation of an explicit
 * grid (f32 [Vz][Vy][Vx], x fastest) at x = clamp(u * V - 0.5, 0, V - 1).
 * Supported shapes are those of cinr_infer_points; the MLP runs in F32 or
 * BF16 (MFMA, FP32 accumulation), encoding and gradients in FP32.
 * ------------------------------------------------------------------------ */
typedef struct cinr_trainer_s* cinr_trainer;

typedef struct {
    int64_t batch;                /* points per step, >= 1 */
    float lr, beta1, beta2, eps;  /* Adam; the step index s uses bias corrections of time s + 1 */
    uint64_t seed;                /* key of the point generator */
    int32_t mlp_dtype;            /* CINR_F32 or CINR_BF16 */
} cinr_train_desc;

/* Size of the caller-provided training workspace (Adam moments, gradients,
 * per-wave partial sums, one batch of points and targets). */
cinr_status cinr_train_workspace_size(cinr_volume vol, const cinr_train_desc* desc, size_t* bytes);
/* Creates a trainer over a caller workspace; zeroes the Adam moments and
 * gradients on `stream`.  The volume must outlive the trainer. */
cinr_status cinr_train_create(cinr_volume vol, const cinr_train_desc* desc, void* d_workspace, size_t ws_bytes,
                              void* stream, cinr_trainer* out);
void cinr_train_destroy(cinr_trainer t);
/* The `batch` points of step `step` into d_u (f32 [batch][3]) and, when
 * d_grid is given (dims grid_dims[3] = Vx, Vy, Vz), their targets into
 * d_target (f32 [batch]). */
cinr_status cinr_train_points(cinr_trainer t, const float* d_grid, const int32_t* grid_dims, int64_t step,
                              float* d_u, float* d_target, void* stream);
/* Loss (f32 [1], nullable) and gradients of n caller points: d_g_table
 * (f32 [entries][F], level-major like the table) and d_g_weights (f32, the
 * weight layout) are overwritten.  Uses the trainer's partial-sum buffer. */
cinr_status cinr_train_gradients(cinr_trainer t, const float* d_u, const float* d_target, int64_t n, float* d_loss,
                                 float* d_g_table, float* d_g_weights, void* stream);
/* One training step: points and targets of `step`, gradients, Adam on the
 * volume's parameters.  d_loss (nullable) receives the batch loss before the
 * update. */
cinr_status cinr_train_step(cinr_trainer t, const float* d_grid, const int32_t* grid_dims, int64_t step,
                            float* d_loss, void* stream);
/* Learning rate of the following steps (for schedules). */
cinr_status cinr_train_set_lr(cinr_trainer t, float lr);
/* Elementwise Adam update of n parameters: m = b1 m + (1-b1) g, v = b2 v +
 * (1-b2) g^2, p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps);
 * step >= 1; the gradient is zeroed afterwards when clear_grad != 0. */
cinr_status cinr_adam_update(float* d_p, float* d_m, float* d_v, float* d_g, int64_t n, int64_t step, float lr,
                             float beta1, float beta2, float eps, int32_t clear_grad, void* stream);

/* Thread-local description of the last failure. */
const char* cinr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
