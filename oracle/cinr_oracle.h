/*
 * cinr_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow CPU reference of the cache-accelerated INR volume renderer of
 * "From Cluster to Desktop: A Cache-Accelerated INR Framework for Interactive
 * Visualization of Tera-Scale Data" (Zavorotny et al.).  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never does.  It shares no code with the GPU path.
 *
 * Two precisions by design:
 *  - value plane (voxel values, colours): FP64;
 *  - decision plane (ray setup, sample positions, LoD choice, brick and
 *    page-table indices): a fixed sequence of correctly rounded binary32
 *    operations (built with -ffp-contract=off, no fast-math), so that page
 *    tables, miss lists and eviction logs can be compared bit for bit.
 */
#ifndef CINR_ORACLE_H
#define CINR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LEVELS 32
#define ORC_MAX_LAYERS 8
#define ORC_MAX_LODS 16
#define ORC_MAX_VOLS 64

/* Hash-grid INR (Section 3, Figure 2): n_levels grids, each a table of
 * T_l = min(2^log2_table, (N_l+1)^3) entries of n_features floats, stored
 * level-major in `table`; then an MLP without biases, ReLU between layers,
 * weights per layer [out][in] row-major, concatenated in `weights`.
 * value = clamp(value_scale * y + value_offset, 0, 1) (Section 4.1). */
typedef struct {
    int32_t dims[3];
    int32_t n_levels, n_features, log2_table;
    int32_t level_res[ORC_MAX_LEVELS];
    int32_t n_layers;
    int32_t widths[ORC_MAX_LAYERS + 1];
    float value_scale, value_offset;
    const float* table;
    const float* weights;
    /* explicit-grid source: when set, the value at voxel coordinate x is the
     * trilinear interpolation of these f32 [Vz][Vy][Vx] samples at x (clamped)
     * instead of the INR, before the same normalisation */
    const float* grid;
} orc_inr;

typedef struct {
    int32_t projection; /* 0 perspective, 1 orthographic */
    int32_t width, height;
    float eye[3], forward[3], right[3], up[3];
    float tan_half_x, tan_half_y, ortho_w, ortho_h;
} orc_camera;

enum { ORC_CACHED = 0, ORC_UNCACHED_DIRECT = 1, ORC_UNCACHED_LATTICE = 2 };

typedef struct {
    float step;          /* sample spacing in LoD-0 voxels */
    float lod_scale;     /* Algorithm 2: LoD distance = |p - eye| * lod_scale */
    float ert_threshold; /* early ray termination at A >= threshold; > 1 disables */
    uint32_t seed;       /* per-run seed of the per-frame stochastic-LoD seed */
    int32_t frame_index;
    int32_t samples_per_iter; /* samples gathered per wavefront step after a true miss */
    int32_t mode;
    int32_t macro_cell;  /* macro-cell side N; 0 = no empty-space skipping */
    const float* macro_minmax; /* [Mz][My][Mx][2] */
    int32_t adapt_max_exp; /* adaptive sampling rate (Section 5.2): < 0 off; else E, the largest step
                              exponent (steps of 2^e sample spacings, e in [0, E]) */
    /* path tracing with Woodcock delta tracking through the same sampler (Section 5.1) */
    int32_t pipeline;      /* 0 = ray marching, 1 = path tracing */
    float pt_density;      /* majorant extinction per LoD-0 voxel; extinction = pt_density * TF opacity */
    float pt_light_dir[3]; /* unit vector toward the directional light */
    float pt_light[3];     /* light term of an unblocked next-event estimate (radiance times phase) */
    float pt_ambient[3];   /* environment radiance seen by scattered rays that leave the box */
    int32_t pt_max_bounces;/* real collisions (scattering events) per path, >= 1 */
    int32_t pt_spp;        /* paths per pixel, >= 1 */
    uint32_t pt_seed;      /* Philox key word 0; word 1 is the frame index */
    /* context-aware LoD (Section 7): with macro-cells, the LoD distance of a
     * sample is scaled by 1 - lod_context * (max - min) of its cell's values,
     * so that cells with a wide value range are sampled at finer LoDs;
     * 0 is the distance-only rule of Algorithm 2 */
    float lod_context;
    /* Performance-mode replay of early ray termination (ray marching): when
     * set, int32 [height][width] holds for every pixel the sample-grid index
     * just past the sample whose compositing ended the ray in the renderer
     * being checked (-1: the ray was not ended early).  The oracle then ends
     * each ray exactly there instead of testing its own opacity, so that every
     * decision of the frame follows the same samples, and counts in
     * orc_stats.ert_violations the replayed ends that its own opacity does not
     * justify: an end where A < threshold - ert_slack, or a sample composited
     * before it where A >= threshold + ert_slack.  NULL: the oracle's own
     * test. */
    const int32_t* ert_replay;
    /* Optional output in the same format: for every pixel, the grid index
     * just past the sample whose compositing ended the ray early, or -1. */
    int32_t* ert_record;
    /* Opacity margin of the replay check: the value error the checked
     * renderer is allowed (its image tolerance); 0 takes 1e-4. */
    double ert_slack;
} orc_params;

/* Events (Philox draws) a pixel may use per frame in path tracing; a pixel
 * that reaches the budget stops: the path in progress is dropped, no further
 * path starts, and the pixel is the mean of the paths it completed. */
#define ORC_PT_MAX_EVENTS 8000

typedef struct {
    int32_t brick;        /* stored brick side B */
    int32_t n_lods;
    int32_t pool_bricks;
    int32_t max_requests;
    int32_t rank_window;  /* ranking clamp above the timestamp (1000) */
    int32_t ranking;      /* 0 = key order of this frame's requests, 1 = priority rank */
    int32_t preload_period; /* frames per LoD step of the coarse-LoD pre-load; 0 = off */
    int32_t pool_f16;     /* nonzero: inserted brick values are rounded to binary16 (a reduced-precision
                             pool, Section 7's future work); 0 = values kept as decoded */
    /* LoD-dependent mixed precision (Section 7's future work): with f16_lods
     * nonzero, bit L set stores LoD L's bricks in the binary16 class of slots
     * [pool_bricks - pool_bricks_f16, pool_bricks) (values rounded to binary16),
     * the other LoDs in the binary32 class of the slots below.  A brick takes
     * a slot of its class only: the class's lowest free slot, else the class's
     * least recently used slot.  Requires pool_f16 = 0, a proper non-empty
     * subset of the LoDs, and max_requests <= the slots of either class. */
    uint32_t f16_lods;
    int32_t pool_bricks_f16;
} orc_cache_desc;

typedef struct {
    int64_t rays, samples, hits, fallbacks, misses, skipped;
    int64_t requested, selected, evicted;
    int64_t ert_violations; /* replayed early terminations not justified by the oracle's opacity */
} orc_stats;

typedef struct orc_cache orc_cache;

/* --- random numbers (published generators) --- */
uint64_t orc_splitmix64(uint64_t state);           /* one output of SplitMix64 from `state` */
uint32_t orc_xorshift32(uint32_t x);               /* one step of Marsaglia's xorshift (13,17,5) */
uint32_t orc_frame_seed(uint32_t seed, uint32_t frame);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* --- INR --- */
int64_t orc_level_size(const orc_inr* m, int level);
int64_t orc_table_entries(const orc_inr* m);
void orc_encode(const orc_inr* m, const double* u, int64_t n, double* feat);
void orc_mlp(const orc_inr* m, const double* feat, int64_t n, double* y);
void orc_value(const orc_inr* m, const double* x, int64_t n, double* v);

/* --- LoD lattice and bricks (Section 4.3.2) --- */
int orc_lod_geometry(const int32_t dims[3], int32_t brick, int32_t n_lods,
                     int32_t* K /*[n_lods][3]*/, int32_t* nb /*[n_lods][3]*/,
                     int64_t* key_offset /*[n_lods+1]*/);
void orc_brick_origin_literal(const int32_t b[3], int32_t lod, int32_t brick, int64_t out[3]);
int orc_decode_bricks(const orc_inr* m, const int32_t* reqs, int64_t n, int32_t brick,
                      int32_t n_lods, double* out);

/* --- macro-cells (Section 5.2) --- */
void orc_macrocells(const orc_inr* m, int32_t cell, float* minmax);
void orc_macrocell_flags(const float* minmax, int64_t n_cells, const float* tf, uint8_t* flags);
/* Step exponent of a cell of maximum opacity mu (> 0): min(E, floor(-log2 mu)),
 * 0 for mu >= 1. */
int32_t orc_step_exp(float mu, int32_t E);
/* Per-cell code of the adaptive sampler: 0xFF for a transparent cell, else
 * its step exponent (orc_step_exp of the cell's maximum opacity). */
void orc_macrocell_step_codes(const float* minmax, int64_t n_cells, const float* tf, int32_t E, uint8_t* codes);

/* --- decision-plane pieces exposed for pinning --- */
int orc_ray_setup(const orc_camera* c, const int32_t dims[3], int32_t i, int32_t j,
                  float o[3], float d[3], float* ts, float* te);
int32_t orc_select_lod(const float p[3], const float eye[3], float lod_scale, uint32_t frame_seed,
                       int32_t lod_floor, int32_t n_lods);
int32_t orc_select_lod_scaled(const float p[3], const float eye[3], float lod_scale, float factor,
                              uint32_t frame_seed, int32_t lod_floor, int32_t n_lods);
int32_t orc_lod_floor(int32_t frame, int32_t period, int32_t n_lods);
/* 1 in the frames of the pre-load whose samples are all forced to the coarsest
 * LoD (frame < period, period > 0): early ray termination is suspended. */
int32_t orc_preload_frame(int32_t frame, int32_t period);

/* --- uncached renderers (no cache state) --- */
int orc_render_uncached(const orc_inr* m, const orc_camera* c, const float* tf,
                        const orc_params* p, double* rgba, orc_stats* st);

/* Listed pixels of a frame against the current residency, no state change. */
int orc_render_pixels(const orc_inr* m, orc_cache* c, const orc_camera* cam, const float* tf, const orc_params* p,
                      const int32_t* pix, int64_t n, double* rgba);

/* --- cached renderer --- */
orc_cache* orc_cache_create(const orc_inr* m, const orc_cache_desc* d);

/* Path tracing primitives (binary32 decision plane).
 * orc_pt_uniform: (r >> 8) * 2^-24, in [0, 1).
 * orc_pt_free_flight: -ln(xi), xi = ((r >> 8) + 1) * 2^-24 in (0, 1], computed
 *   in binary64 and rounded to binary32 (an Exp(1) variate).
 * orc_pt_direction: isotropic direction by Marsaglia's method from the
 *   pixel's events n0, n0+1, ... (Philox counter (pix, n, 0, 0)); returns the
 *   first unused event.
 * orc_pt_segment_exit: distance from p (inside the box [0, vm1]) along d to
 *   the box boundary.
 * orc_tf_alpha32: TF opacity at v in binary32 (rows floor(255 v) and the
 *   next, each interpolation rounded once), clamped to [0, 1]. */
float orc_pt_uniform(uint32_t r);
float orc_pt_free_flight(uint32_t r);
void orc_pt_free_flights(const uint32_t* words, int64_t n, float* out);
uint32_t orc_pt_direction(uint32_t pix, uint32_t n0, const uint32_t key[2], float d[3]);
float orc_pt_segment_exit(const float p[3], const float d[3], const float vm1[3]);
float orc_tf_alpha32(const float* tf, float v);

/* x rounded to the nearest IEEE 754 binary16 value, ties to even (11-bit
 * significand, normal exponents -14..15, subnormal quantum 2^-24), returned
 * as a double; magnitudes that round above 65504 give +-infinity. */
double orc_round_half(double x);
/* A cache shared by n_vols volumes of equal dimensions (ms: array of
 * descriptors); volume v owns keys [v K, (v + 1) K), K = keys of one volume. */
orc_cache* orc_cache_create_multi(const orc_inr* ms, int32_t n_vols, const orc_cache_desc* d);
/* One frame of n views (view i shows volume vol[i]; tfs: n tables of 256x4;
 * rgba: the views' images back to back), then one end-of-frame step. */
int orc_cache_render_views(orc_cache* c, int32_t n, const int32_t* vol, const orc_camera* cams, const float* tfs,
                           const orc_params* ps, double* rgba, orc_stats* sts);
void orc_cache_destroy(orc_cache* c);
int orc_cache_render(orc_cache* c, const orc_camera* cam, const float* tf, const orc_params* p,
                     double* rgba, orc_stats* st);
int orc_cache_prefill(orc_cache* c, const int32_t* keys, int64_t n, int32_t stamp);
int64_t orc_cache_n_keys(const orc_cache* c);
int orc_cache_inject_requests(orc_cache* c, const int32_t* keys, const uint32_t* counts, int64_t n);
int orc_cache_touch(orc_cache* c, int32_t slot, int32_t frame);
int orc_cache_end_frame(orc_cache* c, int32_t frame, orc_stats* st);
void orc_cache_page_table(const orc_cache* c, int32_t* out);
void orc_cache_owner(const orc_cache* c, int32_t* out);
void orc_cache_last_used(const orc_cache* c, int32_t* out);
void orc_cache_rank(const orc_cache* c, int64_t* out);
void orc_cache_req_count(const orc_cache* c, uint32_t* out);
int64_t orc_cache_request_list(const orc_cache* c, int32_t* out);
int64_t orc_cache_miss_list(const orc_cache* c, int32_t* pix_k /*[n][2]*/, float* pos /*[n][3]*/, int64_t cap);
int64_t orc_cache_evict_log(const orc_cache* c, int32_t* out /*[n][4]*/, int64_t cap);
void orc_cache_pool(const orc_cache* c, double* out);
void orc_cache_set_miss_logging(orc_cache* c, int on);
void orc_cache_set_ert_trace(orc_cache* c, int on);
int64_t orc_cache_ert_trace(const orc_cache* c, int32_t* out, int64_t cap);

/* --- training (the learned part) --- */
/* Training batch of `step`: point i is u = (r0, r1, r2) >> 8 * 2^-24 in
 * [0,1)^3, where (r0, r1, r2, r3) = Philox-4x32-10(counter = (i mod 2^32,
 * i >> 32, step mod 2^32, step >> 32), key = (seed mod 2^32, seed >> 32)). */
void orc_train_points(uint64_t seed, int64_t step, int64_t n, double* u /*[n][3]*/);
/* Ground truth of a training point: trilinear interpolation of the explicit
 * grid (f32 [Vz][Vy][Vx], x fastest) at x = clamp(u * V - 0.5, 0, V - 1). */
void orc_grid_trilinear(const float* grid, const int32_t dims[3], const double* u, int64_t n, double* out);

double orc_loss_grad(const orc_inr* m, const double* u, const double* target, int64_t n,
                     double* g_table, double* g_weights);
/* orc_loss_grad with, when bf16_operands != 0, the operands of the hidden
 * layers' products (features, activations, weights, back-propagated errors)
 * rounded to bfloat16 before use; sums and everything else in FP64.  Parity
 * unpinned for bf16_operands != 0: the rounding function is pinned by
 * closed-form values, the placement of the roundings only by reading. */
double orc_loss_grad_prec(const orc_inr* m, const double* u, const double* target, int64_t n,
                          double* g_table, double* g_weights, int bf16_operands);
/* x rounded to binary32 and then to bfloat16, to nearest even. */
double orc_round_bf16(double x);
void orc_adam_step(double* p, double* m1, double* m2, const double* g, int64_t n, int64_t step,
                   double lr, double b1, double b2, double eps);

void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
