// C ABI of libcinr: object lifetimes, argument validation, workspace
// carving and the per-frame launch sequence.  All device work is enqueued on
// the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "frame.h"

using namespace cinr;

namespace {

thread_local std::string g_err;

cinr_status fail(cinr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(CINR_HIP_ERROR, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Sequential carving of a caller workspace.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T>
    T* take(size_t n) {
        T* p = base ? (T*)(base + off) : nullptr;
        off = align256(off + sizeof(T) * (n ? n : 1));
        return p;
    }
};

bool geometry(const int32_t dims[3], int32_t B, int32_t n_lods, CacheGeom& g) {
    if (B < 2 || n_lods < 1 || n_lods > kMaxLods) return false;
    g = CacheGeom{};
    g.brick = B;
    g.div_b1 = make_fastdiv((uint32_t)(B - 1));
    g.n_lods = n_lods;
    int64_t off = 0, doff = 0;
    for (int L = 0; L < n_lods; ++L) {
        int64_t cnt = 1, dcnt = 1;
        for (int a = 0; a < 3; ++a) {
            const int64_t span = (int64_t)dims[a] - 1;
            const int64_t step = (int64_t)1 << L;
            const int64_t K = (span + step - 1) / step + 1;
            const int64_t nb = (K - 1 + (B - 1) - 1) / (B - 1);
            const int64_t dnb = (nb + (1 << kVptShift) - 1) >> kVptShift;
            g.lod[L].K[a] = (int32_t)K;
            g.lod[L].nb[a] = (int32_t)nb;
            if (a < 2) g.lod[L].dnb[a] = (int32_t)dnb;
            cnt *= nb;
            dcnt *= dnb;
        }
        g.lod[L].off = off;
        g.lod[L].doff = doff;
        off += cnt;
        doff += dcnt;
    }
    g.keys_per_vol = off;
    g.dir_per_vol = doff;
    g.n_vols = 1;
    g.n_keys = off;
    return true;
}

}  // namespace

// Per-stage event timing (optional).
struct Timing {
    bool on = false;
    bool march_only = false;  // bracket only the march launches
    std::vector<hipEvent_t> pool;  // free timing events
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        // timestamps only: no system-scope fence (it would write back the
        // L2, full of the march's framebuffer lines, at every record)
        hipEvent_t e = nullptr;
        (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
        return e;
    }
};

// Online tuning of the sampler's launch shape (pipe depth, XCD bands) for one
// image size: the first frames try every candidate twice (results do not
// depend on the shape), the lowest first-march time per sample is kept.
struct SamplerTuner {
    static constexpr int kCand = 24;
    static constexpr int kPipe[kCand] = {1, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 2};
    static constexpr int kBands[kCand] = {1, 1, 4, 4, 16, 16, 1, 1, 4, 4, 16, 16,
                                          1, 1, 4, 4, 16, 16, 1, 1, 4, 4, 16, 16};
    static constexpr int kWaves[kCand] = {3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4};
    // claim direction of the tiles: 1 takes the last tile first (which end
    // holds the tiles of long rays depends on the view)
    static constexpr int kRev[kCand] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr int kRounds = 2;
    // a trial counts when the view's first march left no ray pending (a whole
    // march, as in steady state); after this many frames cut short by true
    // misses, trials count anyway
    static constexpr int kMaxWait = 96;
    int trial = 0;           // frames tried so far
    int waited = 0;          // trial frames not counted
    float ms[kCand] = {};     // sums of first-march time per sample (ns per sample)
    int best = -1;
    hipEvent_t a = nullptr, b = nullptr;
    bool pending = false;    // events of the current trial recorded, not yet read
    // Candidate of trial t: rounds alternate in direction (0..11, then
    // 11..0), so that each candidate's two frames sit symmetrically in the
    // trial window and a trend in the frames' cost (a cache warming up, a
    // pre-load floor dropping) weighs on every candidate alike.
    static int of_trial(int t) {
        const int i = t % kCand;
        return (t / kCand) % 2 == 0 ? i : kCand - 1 - i;
    }
    int cand() const { return best >= 0 ? best : of_trial(trial); }
};

struct cinr_volume_s {
    cinr_volume_desc desc;
    InrDev m;
    int32_t n_cells = 0;
    int32_t M[3] = {0, 0, 0};
    int64_t table_entries = 0;  // hash-table entries over all levels
    int32_t* pinned = nullptr;  // readback of the live-ray counts (one per view)
    FrameVar* stage = nullptr;  // per-frame values of the views (pinned host, read by k_frame_begin)
    hipEvent_t ev = nullptr;     // completion of copies into `pinned` (system-scope fence)
    hipEvent_t ev_nf = nullptr;  // completion of the first marches, which store `pinned` themselves
    Timing timing;
    std::map<uint64_t, SamplerTuner> tuners;  // by image size
    DecodeShape decode_shape;                 // launch shape of this volume's brick decoding
};

namespace {
// Brackets the launches of one stage with timing events when enabled.
struct StageTimer {
    Timing& t;
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(Timing& t_, hipStream_t s_, int stage_) : t(t_), s(s_), stage(stage_) {
        if (t.on && t.march_only && stage != CINR_STAGE_MARCH) return;
        if (t.on) {
            a = t.get();
            (void)hipEventRecord(a, s);
        }
    }
    ~StageTimer() {
        if (a) {
            hipEvent_t b = t.get();
            (void)hipEventRecord(b, s);
            t.recs.push_back(Timing::Rec{stage, a, b});
        }
    }
};
}  // namespace

constexpr int kMaxCacheVols = 64;
constexpr int kMaxViews = 64;

struct cinr_cache_s {
    std::vector<cinr_volume> vols;  // volume v owns keys [v * keys_per_vol, (v + 1) * keys_per_vol)
    cinr_cache_desc desc;
    CacheGeom g;
    CacheDev c;
    InrDev* d_vols = nullptr;  // device copies of the volumes' descriptors
    // side streams of multi-view frames (default priority), created on first use
    static constexpr int kViewStreams = 4;
    hipStream_t vs[kViewStreams] = {};
    hipEvent_t fork = nullptr, join[kViewStreams] = {};
    ~cinr_cache_s() {
        for (int i = 0; i < kViewStreams; ++i) {
            if (vs[i]) (void)hipStreamDestroy(vs[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
        }
        if (fork) (void)hipEventDestroy(fork);
    }
    TopkPlan plan_sel, plan_vic;
    int32_t lim;          // request list length bound: min(max_requests, pool)
    int64_t used_bound[2];  // host upper bounds on occupied slots per class (no LRU pass needed below a class's size)
    int index_of(cinr_volume v) const {
        for (size_t i = 0; i < vols.size(); ++i)
            if (vols[i] == v) return (int)i;
        return -1;
    }
};

// At most n more occupied slots in each class.
static void note_fill(cinr_cache c, int64_t n) {
    c->used_bound[0] = std::min<int64_t>(c->used_bound[0] + n, c->c.split);
    c->used_bound[1] = std::min<int64_t>(c->used_bound[1] + n, c->c.pool_bricks - c->c.split);
}

// ---------------------------------------------------------------------------
// Volume
// ---------------------------------------------------------------------------

extern "C" const char* cinr_last_error(void) { return g_err.c_str(); }

extern "C" cinr_status cinr_create_volume_inr(const cinr_volume_desc* d, cinr_volume* out) {
    if (!d || !out) return fail(CINR_INVALID_ARG, "null argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a)
        if (d->dims[a] < 2 || d->dims[a] > (1 << 24)) return fail(CINR_INVALID_ARG, "dims[%d] = %d out of [2, 2^24]", a, d->dims[a]);
    if (d->n_levels < 1 || d->n_levels > CINR_MAX_LEVELS) return fail(CINR_INVALID_ARG, "n_levels = %d", d->n_levels);
    if (d->n_features < 1 || d->n_features > 4 || d->n_features == 3)
        return fail(CINR_INVALID_ARG, "n_features = %d (1, 2 or 4)", d->n_features);
    if (d->log2_table < 4 || d->log2_table > 30) return fail(CINR_INVALID_ARG, "log2_table = %d", d->log2_table);
    if (d->n_layers < 1 || d->n_layers > CINR_MAX_LAYERS) return fail(CINR_INVALID_ARG, "n_layers = %d", d->n_layers);
    if (d->widths[0] != d->n_levels * d->n_features) return fail(CINR_INVALID_ARG, "widths[0] must be n_levels*n_features");
    if (d->widths[d->n_layers] != 1) return fail(CINR_INVALID_ARG, "the last width must be 1");
    if (!d->d_table || !d->d_weights) return fail(CINR_INVALID_ARG, "null parameter buffer");
    if (d->d_macrocells && d->macrocell_size < 1) return fail(CINR_INVALID_ARG, "macrocell_size must be >= 1");
    cinr_volume v = new cinr_volume_s();
    v->desc = *d;
    InrDev& m = v->m;
    m = InrDev{};
    const uint64_t T = 1ull << d->log2_table;
    uint64_t off = 0;
    for (int a = 0; a < 3; ++a) {
        m.dims[a] = d->dims[a];
        m.vm1[a] = (float)(d->dims[a] - 1);
        m.inv_dims[a] = 1.0 / (double)d->dims[a];
    }
    m.n_levels = d->n_levels;
    m.n_features = d->n_features;
    for (int l = 0; l < d->n_levels; ++l) {
        const int64_t N = d->level_res[l];
        if (N < 1 || N > (1 << 24)) {
            delete v;
            return fail(CINR_INVALID_ARG, "level_res[%d] = %lld", l, (long long)N);
        }
        const uint64_t side = (uint64_t)N + 1;
        const uint64_t dense = side * side * side;
        m.lv[l].res = (double)N;
        m.lv[l].side = (uint32_t)side;
        m.lv[l].side2 = (uint32_t)(side * side <= 0xFFFFFFFFull ? side * side : 0);
        m.lv[l].offset = (uint32_t)off;
        m.lv[l].mask = dense <= T ? 0u : (uint32_t)(T - 1);
        off += dense <= T ? dense : T;
        if (off > 0xFFFFFFFFull) {
            delete v;
            return fail(CINR_INVALID_ARG, "hash table too large");
        }
    }
    v->table_entries = (int64_t)off;
    // the gathers address the table with 32-bit byte offsets
    if (off * (uint64_t)d->n_features * sizeof(float) > 0xFFFFFFFFull) {
        delete v;
        return fail(CINR_INVALID_ARG, "hash table larger than 4 GiB");
    }
    m.value_scale = d->value_scale;
    m.value_offset = d->value_offset;
    m.table = d->d_table;
    m.weights = d->d_weights;
    m.in = d->widths[0];
    m.hidden = d->n_layers == 3 && d->widths[1] == d->widths[2] ? d->widths[1] : -1;
    if (d->d_macrocells) {
        for (int a = 0; a < 3; ++a) v->M[a] = (d->dims[a] + d->macrocell_size - 1) / d->macrocell_size;
        v->n_cells = v->M[0] * v->M[1] * v->M[2];
    }
    *out = v;
    return CINR_OK;
}

extern "C" cinr_status cinr_create_volume_grid(const cinr_grid_desc* d, cinr_volume* out) {
    if (!d || !out || !d->d_grid) return fail(CINR_INVALID_ARG, "null argument");
    for (int a = 0; a < 3; ++a)
        if (d->dims[a] < 2 || d->dims[a] > (1 << 24)) return fail(CINR_INVALID_ARG, "dims[%d] = %d out of [2, 2^24]", a, d->dims[a]);
    if (d->d_macrocells && d->macrocell_size < 1) return fail(CINR_INVALID_ARG, "macrocell_size must be >= 1");
    cinr_volume v = new cinr_volume_s();
    v->desc = cinr_volume_desc{};
    for (int a = 0; a < 3; ++a) v->desc.dims[a] = d->dims[a];
    v->desc.value_scale = d->value_scale;
    v->desc.value_offset = d->value_offset;
    v->desc.d_macrocells = d->d_macrocells;
    v->desc.macrocell_size = d->macrocell_size;
    InrDev& m = v->m;
    m = InrDev{};
    for (int a = 0; a < 3; ++a) {
        m.dims[a] = d->dims[a];
        m.vm1[a] = (float)(d->dims[a] - 1);
        m.inv_dims[a] = 1.0 / (double)d->dims[a];
    }
    m.value_scale = d->value_scale;
    m.value_offset = d->value_offset;
    m.hidden = -1;
    m.grid = d->d_grid;
    if (d->d_macrocells) {
        for (int a = 0; a < 3; ++a) v->M[a] = (d->dims[a] + d->macrocell_size - 1) / d->macrocell_size;
        v->n_cells = v->M[0] * v->M[1] * v->M[2];
    }
    *out = v;
    return CINR_OK;
}

extern "C" void cinr_destroy_volume(cinr_volume v) {
    if (!v) return;
    if (v->pinned) (void)hipHostFree(v->pinned);
    if (v->stage) (void)hipHostFree(v->stage);
    if (v->ev) (void)hipEventDestroy(v->ev);
    if (v->ev_nf) (void)hipEventDestroy(v->ev_nf);
    for (auto& r : v->timing.recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : v->timing.pool) (void)hipEventDestroy(e);
    delete v;
}

extern "C" cinr_status cinr_set_timing(cinr_volume v, int32_t enable) {
    if (!v) return fail(CINR_INVALID_ARG, "null volume");
    if (enable < 0 || enable > 2) return fail(CINR_INVALID_ARG, "timing mode %d (0, 1 or 2)", enable);
    v->timing.on = enable != 0;
    v->timing.march_only = enable == 2;
    return CINR_OK;
}

extern "C" cinr_status cinr_collect_timing(cinr_volume v, double* ms, int64_t* launches) {
    if (!v || !ms || !launches) return fail(CINR_INVALID_ARG, "null argument");
    for (int i = 0; i < CINR_STAGE_COUNT; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    Timing& t = v->timing;
    if (!t.recs.empty()) HIP_TRY(hipEventSynchronize(t.recs.back().b));
    for (auto& r : t.recs) {
        float e = 0.0f;
        HIP_TRY(hipEventElapsedTime(&e, r.a, r.b));
        ms[r.stage] += e;
        launches[r.stage] += 1;
        t.pool.push_back(r.a);
        t.pool.push_back(r.b);
    }
    t.recs.clear();
    return CINR_OK;
}

extern "C" cinr_status cinr_lod_geometry(cinr_volume v, int32_t brick, int32_t n_lods, int32_t* nb, int64_t* key_offset) {
    if (!v) return fail(CINR_INVALID_ARG, "null volume");
    CacheGeom g;
    if (!geometry(v->desc.dims, brick, n_lods, g)) return fail(CINR_INVALID_ARG, "brick >= 2 and 1 <= n_lods <= 16 required");
    for (int L = 0; L < n_lods; ++L) {
        if (nb)
            for (int a = 0; a < 3; ++a) nb[3 * L + a] = g.lod[L].nb[a];
        if (key_offset) key_offset[L] = g.lod[L].off;
    }
    if (key_offset) key_offset[n_lods] = g.n_keys;
    return CINR_OK;
}

static cinr_status check_shape(cinr_volume v, int32_t prec) {
    if (prec != CINR_F32 && prec != CINR_BF16 && prec != CINR_F16 && prec != CINR_BF16X3)
        return fail(CINR_INVALID_ARG, "mlp_dtype = %d", prec);
    if (v->m.grid) return CINR_OK;
    if (v->m.hidden < 0 || !inr_shape_supported(v->m))
        return fail(CINR_UNSUPPORTED, "no gfx950 kernel for this INR shape (3 layers, levels x features in {8x2, 16x2, 16x4}, hidden 32 or 64)");
    return CINR_OK;
}

extern "C" cinr_status cinr_infer_points(cinr_volume v, const float* d_pos, int64_t n, float* d_out, int32_t prec, void* stream) {
    if (!v || (n > 0 && (!d_pos || !d_out)) || n < 0) return fail(CINR_INVALID_ARG, "invalid arguments");
    cinr_status st = check_shape(v, prec);
    if (st) return st;
    HIP_TRY(inr_infer_points(v->m, d_pos, n, d_out, prec, (hipStream_t)stream));
    return CINR_OK;
}

namespace {
cinr_status check_decode_shape(int32_t brick, int32_t parts, int32_t stage_kib, DecodeShape* out) {
    if (parts != 0 && parts != 1 && parts != 2 && parts != 4 && parts != 8 && parts != 16)
        return fail(CINR_INVALID_ARG, "parts_per_brick = %d (0, 1, 2, 4, 8 or 16)", parts);
    if (parts > 0 && stage_kib != 0 && stage_kib != 32 && stage_kib != 64)
        return fail(CINR_INVALID_ARG, "stage_kib = %d (0, 32 or 64)", stage_kib);
    if (parts > 0 && brick > 0 && brick % parts != 0)
        return fail(CINR_INVALID_ARG, "brick %d is not a multiple of parts_per_brick %d", brick, parts);
    out->parts = parts;
    out->stage_floats = parts > 0 ? stage_kib * 256 : 0;
    return CINR_OK;
}

cinr_status decode_with(cinr_volume v, const int32_t* d_reqs, int32_t n, int32_t brick, float* d_out, int32_t prec,
                        DecodeShape shape, void* stream) {
    if (!v || n < 0 || (n > 0 && (!d_reqs || !d_out))) return fail(CINR_INVALID_ARG, "invalid arguments");
    if (brick < 2 || brick > 64) return fail(CINR_INVALID_ARG, "brick = %d out of [2, 64]", brick);
    cinr_status st = check_shape(v, prec);
    if (st) return st;
    CacheGeom g;
    geometry(v->desc.dims, brick, kMaxLods, g);
    const BrickOut out{d_out, nullptr, 0x7FFFFFFF};
    if (brick % (shape.parts > 0 ? shape.parts : 1) != 0) shape = DecodeShape{};
    HIP_TRY(inr_decode_bricks(v->m, g, d_reqs, nullptr, nullptr, n, nullptr, out, prec, (hipStream_t)stream, shape));
    return CINR_OK;
}
}  // namespace

extern "C" cinr_status cinr_decode_bricks(cinr_volume v, const int32_t* d_reqs, int32_t n, int32_t brick, float* d_out,
                                          int32_t prec, void* stream) {
    if (!v) return fail(CINR_INVALID_ARG, "invalid arguments");
    return decode_with(v, d_reqs, n, brick, d_out, prec, v->decode_shape, stream);
}

extern "C" cinr_status cinr_decode_bricks_shaped(cinr_volume v, const int32_t* d_reqs, int32_t n, int32_t brick,
                                                 float* d_out, int32_t prec, int32_t parts, int32_t stage_kib,
                                                 void* stream) {
    DecodeShape shape;
    cinr_status st = check_decode_shape(brick, parts, stage_kib, &shape);
    if (st) return st;
    return decode_with(v, d_reqs, n, brick, d_out, prec, shape, stream);
}

namespace {
// Candidate launch shapes of brick decoding (parts per brick, stage KiB),
// in the order cinr_tune_decode reports their times.
constexpr int kDecodeCand = 16;
constexpr int32_t kDecodeParts[kDecodeCand] = {0, 1, 1, 1, 2, 2, 2, 4, 4, 4, 8, 8, 8, 16, 16, 16};
constexpr int32_t kDecodeKib[kDecodeCand] = {0, 0, 32, 64, 0, 32, 64, 0, 32, 64, 0, 32, 64, 0, 32, 64};
}  // namespace

extern "C" cinr_status cinr_tune_decode(cinr_volume v, const int32_t* d_reqs, int32_t n, int32_t brick, float* d_out,
                                        int32_t prec, int32_t reps, float* ms_out, int32_t* chosen, void* stream) {
    if (!v || n < 1 || !d_reqs || !d_out || reps < 1) return fail(CINR_INVALID_ARG, "invalid arguments");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    int best = -1;
    float best_ms = 0.0f;
    cinr_status st = CINR_OK;
    for (int i = 0; i < kDecodeCand && st == CINR_OK; ++i) {
        float ms = -1.0f;
        if (kDecodeParts[i] == 0 || brick % kDecodeParts[i] == 0) {
            DecodeShape shape;
            st = check_decode_shape(brick, kDecodeParts[i], kDecodeKib[i], &shape);
            if (st == CINR_OK) st = decode_with(v, d_reqs, n, brick, d_out, prec, shape, stream);  // warm-up
            if (st == CINR_OK && hipEventRecord(a, s) != hipSuccess) st = fail(CINR_HIP_ERROR, "event record");
            for (int r = 0; r < reps && st == CINR_OK; ++r) st = decode_with(v, d_reqs, n, brick, d_out, prec, shape, stream);
            if (st == CINR_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                                  hipEventElapsedTime(&ms, a, b) != hipSuccess))
                st = fail(CINR_HIP_ERROR, "decode timing");
            if (st == CINR_OK) {
                ms /= (float)reps;
                if (best < 0 || ms < best_ms) {
                    best = i;
                    best_ms = ms;
                }
            }
        }
        if (ms_out) ms_out[i] = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st) return st;
    DecodeShape shape;
    check_decode_shape(brick, kDecodeParts[best], kDecodeKib[best], &shape);
    v->decode_shape = shape;
    if (chosen) *chosen = best;
    return CINR_OK;
}

extern "C" cinr_status cinr_set_decode_shape(cinr_volume v, int32_t parts, int32_t stage_kib) {
    if (!v) return fail(CINR_INVALID_ARG, "null volume");
    DecodeShape shape;
    cinr_status st = check_decode_shape(0, parts, stage_kib, &shape);
    if (st) return st;
    v->decode_shape = shape;
    return CINR_OK;
}

extern "C" cinr_status cinr_build_macrocells(cinr_volume v, int32_t cell, float* d_minmax, int32_t prec, void* stream) {
    if (!v || cell < 1 || !d_minmax) return fail(CINR_INVALID_ARG, "invalid arguments");
    cinr_status st = check_shape(v, prec);
    if (st) return st;
    HIP_TRY(inr_macrocells(v->m, cell, d_minmax, prec, (hipStream_t)stream));
    return CINR_OK;
}

// ---------------------------------------------------------------------------
// Cache
// ---------------------------------------------------------------------------

static cinr_status check_cache_desc(const cinr_volume* vols, int32_t n_vols, const cinr_cache_desc* d, CacheGeom& g) {
    if (!vols || !d) return fail(CINR_INVALID_ARG, "null argument");
    if (n_vols < 1 || n_vols > kMaxCacheVols) return fail(CINR_INVALID_ARG, "%d volumes (1 to %d)", n_vols, kMaxCacheVols);
    for (int i = 0; i < n_vols; ++i) {
        const cinr_volume v = vols[i];
        if (!v) return fail(CINR_INVALID_ARG, "null volume %d", i);
        const InrDev& a = vols[0]->m;
        const InrDev& b = v->m;
        for (int k = 0; k < 3; ++k)
            if (b.dims[k] != a.dims[k]) return fail(CINR_INVALID_ARG, "volume %d: dimensions differ from volume 0", i);
        if ((a.grid == nullptr) != (b.grid == nullptr) ||
            (!a.grid && (a.n_levels != b.n_levels || a.n_features != b.n_features || a.in != b.in || a.hidden != b.hidden)))
            return fail(CINR_INVALID_ARG, "volume %d: shape differs from volume 0 (a shared cache decodes all volumes in one launch)", i);
    }
    if (d->brick < 2 || d->brick > 64) return fail(CINR_INVALID_ARG, "brick = %d out of [2, 64]", d->brick);
    if (d->n_lods < 1 || d->n_lods > CINR_MAX_LODS) return fail(CINR_INVALID_ARG, "n_lods = %d", d->n_lods);
    if (d->pool_bricks < 0 || d->max_requests < 0 || d->max_requests > kMaxRequests)
        return fail(CINR_INVALID_ARG, "pool_bricks >= 0 and 0 <= max_requests <= %d required", kMaxRequests);
    if (d->rank_window < 0) return fail(CINR_INVALID_ARG, "rank_window < 0");
    if (d->miss_log_capacity < 0 || d->evict_log_capacity < 0) return fail(CINR_INVALID_ARG, "negative log capacity");
    if (d->pool_dtype != CINR_F32 && d->pool_dtype != CINR_F16)
        return fail(CINR_INVALID_ARG, "pool_dtype = %d (CINR_F32 or CINR_F16)", d->pool_dtype);
    if (d->f16_lods != 0u) {
        const uint32_t all = d->n_lods >= 32 ? 0xFFFFFFFFu : (1u << d->n_lods) - 1u;
        if (d->pool_dtype != CINR_F32)
            return fail(CINR_INVALID_ARG, "f16_lods: the classes of a mixed pool need pool_dtype = CINR_F32");
        if ((d->f16_lods & ~all) || d->f16_lods == all)
            return fail(CINR_INVALID_ARG, "f16_lods = 0x%x: a proper subset of the %d LoDs", d->f16_lods, d->n_lods);
        const int32_t p16 = d->pool_bricks_f16, p32 = d->pool_bricks - d->pool_bricks_f16;
        if (p16 < 1 || p32 < 1 || d->max_requests > p16 || d->max_requests > p32)
            return fail(CINR_INVALID_ARG, "pool_bricks_f16 = %d of %d: each class needs max_requests (%d) slots or more",
                        p16, d->pool_bricks, d->max_requests);
    }
    if (d->virtual_page_table != 0 && d->virtual_page_table != 1)
        return fail(CINR_INVALID_ARG, "virtual_page_table = %d (0 or 1)", d->virtual_page_table);
    if (d->pt_blocks < 0) return fail(CINR_INVALID_ARG, "pt_blocks < 0");
    if (!geometry(vols[0]->desc.dims, d->brick, d->n_lods, g)) return fail(CINR_INVALID_ARG, "invalid geometry");
    g.n_vols = n_vols;
    g.n_keys = g.keys_per_vol * n_vols;
    if (g.n_keys > 0x7FFFFFFF) return fail(CINR_UNSUPPORTED, "more than 2^31 bricks");
    return CINR_OK;
}

static size_t cache_layout(const cinr_cache_desc* d, const CacheGeom& g, CacheDev* c, TopkPlan* ps, TopkPlan* pv,
                           void* base, InrDev** vols_out = nullptr) {
    const int64_t nk = g.n_keys;
    const int32_t P = d->pool_bricks;
    const int32_t lim = std::max(1, std::min(d->max_requests, P));
    const int32_t ins_cap = std::max(lim, (int32_t)std::min<int64_t>(P, nk));
    const TopkPlan plan_sel = make_topk_plan(nk, lim);
    const TopkPlan plan_vic = make_topk_plan(P > 0 ? P : 1, lim);
    size_t buf = 0;
    for (const TopkPlan* p : {&plan_sel, &plan_vic})
        for (int i = 0; i < p->n_pass; ++i) buf = std::max(buf, (size_t)p->blocks[i] * lim);
    Carver cv(base);
    CacheDev x{};
    const bool virt = d->virtual_page_table != 0;
    x.pt = virt ? nullptr : cv.take<int32_t>(nk);
    if (virt) {
        // directory over all volumes, block pool (never short at its bound:
        // a block in use holds at least one of the pool's bricks)
        const int64_t nd = g.dir_per_vol * g.n_vols;
        const int64_t bound = std::max<int64_t>(1, std::min<int64_t>(nd, P));
        const int64_t cap = d->pt_blocks > 0 ? std::min<int64_t>(d->pt_blocks, bound) : bound;
        x.vdir = cv.take<int32_t>(nd);
        x.vblk = cv.take<int32_t>((size_t)cap * kVptEntries);
        x.vcnt = cv.take<int32_t>(cap);
        x.vfree = cv.take<int32_t>(cap);
        x.vcap = (int32_t)cap;
    }
    x.rank = cv.take<int64_t>(nk);
    x.req = cv.take<uint32_t>(nk);
    x.last_req = d->keep_request_counts ? cv.take<uint32_t>(nk) : nullptr;
    x.touched = cv.take<int32_t>(nk);
    x.cand = cv.take<uint64_t>(nk);
    x.owner = cv.take<int32_t>(P);
    x.last_used = cv.take<int32_t>(P);
    x.ins_keys = cv.take<int32_t>(ins_cap);
    x.ins_slots = cv.take<int32_t>(ins_cap);
    x.ins_reqs = cv.take<int32_t>((size_t)ins_cap * 4);
    x.ins_vols = cv.take<int32_t>(ins_cap);
    x.ins_old = cv.take<int32_t>(ins_cap);
    x.topk[0] = cv.take<uint64_t>(buf);
    x.topk[1] = cv.take<uint64_t>(buf);
    x.sel = cv.take<uint64_t>(lim);
    x.vic = cv.take<uint64_t>(lim);
    x.vic1 = cv.take<uint64_t>(lim);
    x.misslog = cv.take<MissLogRec>(d->miss_log_capacity);
    x.misslog_cap = d->miss_log_capacity;
    x.evlog = cv.take<int32_t>((size_t)d->evict_log_capacity * 4);
    x.evlog_cap = d->evict_log_capacity;
    x.ctr = cv.take<CacheCtr>(1);
    x.views = cv.take<ViewEnd>(kMaxFrameViews);
    if (vols_out) *vols_out = cv.take<InrDev>(g.n_vols);
    x.pool_bricks = P;
    x.max_requests = d->max_requests;
    x.rank_window = d->rank_window;
    x.ranking = d->ranking;
    x.ins_cap = ins_cap;
    if (!d->keep_request_counts && base == nullptr) x.last_req = nullptr;
    if (c) *c = x;
    if (ps) *ps = plan_sel;
    if (pv) *pv = plan_vic;
    return cv.off;
}

extern "C" cinr_status cinr_cache_workspace_size_multi(const cinr_volume* vols, int32_t n_vols, const cinr_cache_desc* d,
                                                     size_t* bytes) {
    CacheGeom g;
    cinr_status st = check_cache_desc(vols, n_vols, d, g);
    if (st) return st;
    if (!bytes) return fail(CINR_INVALID_ARG, "null bytes");
    InrDev* unused = nullptr;
    *bytes = cache_layout(d, g, nullptr, nullptr, nullptr, nullptr, &unused);
    return CINR_OK;
}

extern "C" cinr_status cinr_cache_workspace_size(cinr_volume v, const cinr_cache_desc* d, size_t* bytes) {
    return cinr_cache_workspace_size_multi(&v, 1, d, bytes);
}

extern "C" cinr_status cinr_create_cache_multi(const cinr_volume* vols, int32_t n_vols, const cinr_cache_desc* d,
                                               void* d_pool, size_t pool_bytes, void* d_ws, size_t ws_bytes,
                                               void* stream, cinr_cache* out) {
    if (!out) return fail(CINR_INVALID_ARG, "null out");
    *out = nullptr;
    CacheGeom g;
    cinr_status st = check_cache_desc(vols, n_vols, d, g);
    if (st) return st;
    const size_t B3 = (size_t)d->brick * d->brick * d->brick;
    const int32_t split = d->f16_lods ? d->pool_bricks - d->pool_bricks_f16 : d->pool_bricks;
    const size_t bytes32 = d->pool_dtype == CINR_F16 ? 0 : (size_t)split * B3 * 4;
    const size_t pool_need = d->pool_dtype == CINR_F16 ? (size_t)d->pool_bricks * B3 * 2
                                                       : bytes32 + (size_t)(d->pool_bricks - split) * B3 * 2;
    if (pool_bytes < pool_need) return fail(CINR_OUT_OF_MEMORY, "pool of %zu bytes < %zu needed", pool_bytes, pool_need);
    if (d->pool_bricks > 0 && !d_pool) return fail(CINR_INVALID_ARG, "null pool");
    InrDev* unused = nullptr;
    const size_t need = cache_layout(d, g, nullptr, nullptr, nullptr, nullptr, &unused);
    if (!d_ws || ws_bytes < need) return fail(CINR_OUT_OF_MEMORY, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    cinr_cache c = new cinr_cache_s();
    c->vols.assign(vols, vols + n_vols);
    c->desc = *d;
    c->g = g;
    cache_layout(d, g, &c->c, &c->plan_sel, &c->plan_vic, d_ws, &c->d_vols);
    c->c.pool = d_pool;
    c->c.pool_kind = d->f16_lods ? POOL_MIXED : (d->pool_dtype == CINR_F16 ? POOL_F16 : POOL_F32);
    c->c.split = split;
    c->c.f16_lods = d->f16_lods;
    c->c.pool16 = d->f16_lods ? (void*)((char*)d_pool + bytes32) : nullptr;
    c->lim = std::max(1, std::min(d->max_requests, d->pool_bricks));
    c->used_bound[0] = c->used_bound[1] = 0;
    hipStream_t s = (hipStream_t)stream;
    std::vector<InrDev> host(n_vols);
    for (int i = 0; i < n_vols; ++i) host[i] = vols[i]->m;
    hipError_t e = launch_cache_init(c->c, g.n_keys, g.dir_per_vol * g.n_vols, s);
    // the copy is staged from pageable memory before the call returns
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_vols, host.data(), sizeof(InrDev) * n_vols, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        delete c;
        return fail(CINR_HIP_ERROR, "cache init: %s", hipGetErrorString(e));
    }
    *out = c;
    return CINR_OK;
}

extern "C" cinr_status cinr_create_cache(cinr_volume v, const cinr_cache_desc* d, void* d_pool, size_t pool_bytes,
                                         void* d_ws, size_t ws_bytes, void* stream, cinr_cache* out) {
    return cinr_create_cache_multi(&v, 1, d, d_pool, pool_bytes, d_ws, ws_bytes, stream, out);
}

// Decoding of the bricks selected for insertion (at most n_cap of them;
// none unless *gate != 0 when a gate is given).
static hipError_t decode_selected(cinr_cache c, int32_t n_cap, int32_t prec, const uint32_t* gate, hipStream_t s) {
    const CacheDev& cd = c->c;
    BrickOut out{cd.pool, cd.pool16, cd.split};
    if (cd.pool_kind == POOL_F16) {
        out.out16 = cd.pool;
        out.split = 0;
    }
    if (c->vols.size() == 1)
        return inr_decode_bricks(c->vols[0]->m, c->g, cd.ins_reqs, &cd.ctr->n_sel, gate, n_cap, cd.ins_slots, out,
                                 prec, s, c->vols[0]->decode_shape);
    return inr_decode_bricks_multi(c->d_vols, c->vols[0]->m, c->g, cd.ins_reqs, cd.ins_vols, &cd.ctr->n_sel, gate,
                                   n_cap, cd.ins_slots, out, prec, s, c->vols[0]->decode_shape);
}

extern "C" void cinr_destroy_cache(cinr_cache c) { delete c; }

extern "C" cinr_status cinr_cache_prefill(cinr_cache c, const int32_t* d_keys, int32_t n, int32_t stamp, int32_t prec,
                                          void* stream) {
    if (!c || n < 0 || (n > 0 && !d_keys)) return fail(CINR_INVALID_ARG, "invalid arguments");
    if (n > c->c.ins_cap) return fail(CINR_INVALID_ARG, "prefill of %d bricks exceeds %d", n, c->c.ins_cap);
    cinr_status st = check_shape(c->vols[0], prec);
    if (st) return st;
    if (n == 0) return CINR_OK;
    hipStream_t s = (hipStream_t)stream;
    note_fill(c, n);
    HIP_TRY(launch_prefill_setup(c->c, c->g, d_keys, n, stamp, s));
    HIP_TRY(launch_insert(c->c, c->g, n, nullptr, s));
    if (c->c.vdir) HIP_TRY(launch_vpt_update(c->c, c->g, nullptr, s));
    HIP_TRY(decode_selected(c, n, prec, nullptr, s));
    return CINR_OK;
}

// ---------------------------------------------------------------------------
// Render
// ---------------------------------------------------------------------------

struct RenderLayout {
    int32_t* live0;
    int32_t* live1;
    int32_t* k_next;
    int32_t* pend_pix;
    int32_t* pend_n;
    float* vals;
    float4* miss_rec;
    IterCtr* ctr;
    uint32_t* claim;
    uint64_t* flags;
    unsigned long long* stats;
    FrameVar* var;
    uint32_t* gate;  // frame-end gate (view 0's is the frame's)
    uint32_t* ticket;  // finished workgroups of the first march (fused gather)
    uint8_t* cell_code;  // adaptive sampling: per macro-cell step codes
    uint8_t* vexp;       // adaptive sampling: step exponent of each gathered sample
    PtState* pts;        // path tracing: per-pixel path state (null for ray marching)
};

static size_t render_layout(int64_t npix, int32_t S, int64_t n_cells, bool path, RenderLayout* r, void* base) {
    Carver cv(base);
    RenderLayout x;
    x.live0 = cv.take<int32_t>(npix);
    x.live1 = cv.take<int32_t>(npix);
    x.k_next = cv.take<int32_t>(npix);
    x.pend_pix = cv.take<int32_t>(npix);
    x.pend_n = cv.take<int32_t>(npix);
    x.vals = cv.take<float>((size_t)npix * S);
    x.miss_rec = cv.take<float4>((size_t)npix * S);
    x.ctr = cv.take<IterCtr>(kMaxIters + 2);
    x.claim = cv.take<uint32_t>(16 * kClaimStride);
    x.flags = cv.take<uint64_t>((size_t)(n_cells + 63) / 64);
    x.stats = cv.take<unsigned long long>(ST_COUNT);
    x.var = cv.take<FrameVar>(1);
    x.gate = cv.take<uint32_t>(1);
    x.ticket = cv.take<uint32_t>(1);
    x.cell_code = cv.take<uint8_t>((size_t)(n_cells > 0 ? n_cells : 1));
    x.vexp = cv.take<uint8_t>((size_t)npix * S);
    x.pts = path ? cv.take<PtState>((size_t)npix) : nullptr;
    if (r) *r = x;
    return cv.off;
}

// Pixels of a path-traced image: the inference writes into the path state at
// 32-bit word indices pixel * 32 + k.
constexpr int64_t kMaxPathPixels = int64_t(1) << 27;

extern "C" cinr_status cinr_render_workspace_size(cinr_volume v, int32_t W, int32_t H, int32_t S, size_t* bytes) {
    if (!v || !bytes || W < 1 || H < 1 || S < 1 || S > 64) return fail(CINR_INVALID_ARG, "invalid arguments");
    if ((int64_t)W * H * S > 0xFFFFFFFFll) return fail(CINR_INVALID_ARG, "width*height*samples_per_iter >= 2^32");
    *bytes = render_layout((int64_t)W * H, S, v->n_cells, false, nullptr, nullptr);
    return CINR_OK;
}

extern "C" cinr_status cinr_path_workspace_size(cinr_volume v, int32_t W, int32_t H, int32_t S, size_t* bytes) {
    if (!v || !bytes || W < 1 || H < 1 || S < 1 || S > 64) return fail(CINR_INVALID_ARG, "invalid arguments");
    if ((int64_t)W * H >= kMaxPathPixels) return fail(CINR_INVALID_ARG, "width*height >= 2^27 for the path tracer");
    if ((int64_t)W * H * S > 0xFFFFFFFFll) return fail(CINR_INVALID_ARG, "width*height*samples_per_iter >= 2^32");
    *bytes = render_layout((int64_t)W * H, S, v->n_cells, true, nullptr, nullptr);
    return CINR_OK;
}

extern "C" cinr_status cinr_pt_free_flight(const uint32_t* d_words, int64_t n, float* d_out, void* stream) {
    if (n < 0 || (n > 0 && (!d_words || !d_out))) return fail(CINR_INVALID_ARG, "invalid arguments");
    HIP_TRY(launch_pt_free_flight(d_words, n, d_out, (hipStream_t)stream));
    return CINR_OK;
}

namespace {

// One view of a frame: its volume, descriptor and workspace, and the state of
// its wavefront iterations.
struct ViewRun {
    cinr_volume v = nullptr;
    hipStream_t st = nullptr;  // stream of this view's launches
    FrameDev f{};
    FrameVar hv{};              // this frame's camera, index and LoD seed (host copy)
    FrameVar* stage = nullptr;  // pinned host block that k_frame_begin reads hv from
    RenderLayout L{};
    int64_t npix = 0, max_iters = 0, queued = 0;
    int32_t prec = 0;
    int n_iters = 0;
    bool live = true;       // iterations left
    SamplerTuner* tuner = nullptr;
    bool timing_trial = false;
};

cinr_status check_camera(const cinr_camera* cam) {
    if (cam->width < 1 || cam->height < 1) return fail(CINR_INVALID_ARG, "empty image");
    if (cam->projection != CINR_PERSPECTIVE && cam->projection != CINR_ORTHOGRAPHIC)
        return fail(CINR_INVALID_ARG, "projection = %d", cam->projection);
    const float* vs[4] = {cam->eye, cam->forward, cam->right, cam->up};
    for (const float* q : vs)
        for (int a = 0; a < 3; ++a)
            if (!isfinite(q[a])) return fail(CINR_INVALID_ARG, "non-finite camera vector");
    const float sc[4] = {cam->tan_half_x, cam->tan_half_y, cam->ortho_w, cam->ortho_h};
    for (float x : sc)
        if (!isfinite(x)) return fail(CINR_INVALID_ARG, "non-finite camera extent");
    if (cam->forward[0] == 0.0f && cam->forward[1] == 0.0f && cam->forward[2] == 0.0f)
        return fail(CINR_INVALID_ARG, "zero forward vector");
    return CINR_OK;
}

// Per-frame values of a view: camera, frame index, and the per-frame seed and
// LoD floor of the cached mode (Sec. 4.3.4 pre-load, Sec. 5.3 seed).
FrameVar frame_var(cinr_cache c, const cinr_camera* cam, const cinr_render_params* rp) {
    FrameVar h{};
    h.cam.proj = cam->projection;
    h.cam.W = cam->width;
    h.cam.H = cam->height;
    for (int a = 0; a < 3; ++a) {
        h.cam.eye[a] = cam->eye[a];
        h.cam.fwd[a] = cam->forward[a];
        h.cam.right[a] = cam->right[a];
        h.cam.up[a] = cam->up[a];
    }
    h.cam.tanx = cam->tan_half_x;
    h.cam.tany = cam->tan_half_y;
    h.cam.ow = cam->ortho_w;
    h.cam.oh = cam->ortho_h;
    h.frame = rp->frame_index;
    if (c) {
        // per-frame seed of the stochastic LoD: high half of SplitMix64 of (seed << 32 | frame)
        uint64_t z = (((uint64_t)rp->seed << 32) | (uint64_t)(uint32_t)rp->frame_index) + 0x9e3779b97f4a7c15ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z = z ^ (z >> 31);
        h.frame_seed = (uint32_t)(z >> 32);
        int32_t floor_ = 0;
        if (c->desc.preload_period > 0) {
            floor_ = c->desc.n_lods - 1 - rp->frame_index / c->desc.preload_period;
            if (floor_ < 0) floor_ = 0;
        }
        h.lod_floor = floor_;
        // the frames that force the coarsest LoD march without early ray
        // termination, so that the coarsest bricks behind opaque material
        // are requested too (Sec. 4.3.4: a low-resolution copy of nearly the
        // whole volume to fall back on)
        h.preload = c->desc.preload_period > 0 && rp->frame_index < c->desc.preload_period ? 1 : 0;
    }
    return h;
}

// Validates one view and fills its frame descriptor.
// Without `trials`, a view whose launch shape is left to the tuner takes the
// shape already tuned for its image size, else the first candidate, and no
// trial is timed.
cinr_status prepare_view(cinr_cache c, cinr_volume v, const cinr_camera* cam, const float* d_tf,
                         const cinr_render_params* rp, float* d_rgba, cinr_frame_stats* d_stats, void* d_ws,
                         size_t ws_bytes, ViewRun& r, bool trials = true) {
    if (!v || !cam || !d_tf || !rp || !d_rgba) return fail(CINR_INVALID_ARG, "null argument");
    cinr_status st = check_camera(cam);
    if (st) return st;
    if (rp->mode != CINR_CACHED && rp->mode != CINR_UNCACHED_DIRECT && rp->mode != CINR_UNCACHED_LATTICE)
        return fail(CINR_INVALID_ARG, "mode = %d", rp->mode);
    if (!(rp->step > 0.0f) || !isfinite(rp->step)) return fail(CINR_INVALID_ARG, "step must be > 0");
    if (!(rp->lod_scale >= 0.0f)) return fail(CINR_INVALID_ARG, "lod_scale must be >= 0");
    if (rp->pipe_depth != 0 && rp->pipe_depth != 1 && rp->pipe_depth != 2 && rp->pipe_depth != 4 && rp->pipe_depth != 8)
        return fail(CINR_INVALID_ARG, "pipe_depth must be 0, 1, 2, 4 or 8");
    if (rp->xcd_bands < 0 || rp->xcd_bands > 64) return fail(CINR_INVALID_ARG, "xcd_bands must be in [0, 64]");
    if (rp->waves_per_simd != 0 && rp->waves_per_simd != 3 && rp->waves_per_simd != 4)
        return fail(CINR_INVALID_ARG, "waves_per_simd must be 0, 3 or 4");
    if (rp->samples_per_iter < 1 || rp->samples_per_iter > 64)
        return fail(CINR_INVALID_ARG, "samples_per_iter must be in [1, 64]");
    if (rp->adapt_max_exp < 0 || rp->adapt_max_exp > 14)
        return fail(CINR_INVALID_ARG, "adapt_max_exp must be in [0, 14]");
    if (!(rp->lod_context >= 0.0f && rp->lod_context <= 1.0f))
        return fail(CINR_INVALID_ARG, "lod_context must be in [0, 1]");
    if (rp->pipeline != CINR_RAY_MARCH && rp->pipeline != CINR_PATH_TRACE)
        return fail(CINR_INVALID_ARG, "pipeline = %d", rp->pipeline);
    const bool path = rp->pipeline == CINR_PATH_TRACE;
    if (path) {
        if (!(rp->pt_density > 0.0f) || !isfinite(rp->pt_density)) return fail(CINR_INVALID_ARG, "pt_density must be > 0");
        if (rp->pt_max_bounces < 1) return fail(CINR_INVALID_ARG, "pt_max_bounces must be >= 1");
        if (rp->pt_spp < 1 || rp->pt_spp > 65535) return fail(CINR_INVALID_ARG, "pt_spp must be in [1, 65535]");
        if (rp->adapt_max_exp != 0) return fail(CINR_INVALID_ARG, "the path tracer has no adaptive sampling rate");
        for (int a = 0; a < 3; ++a)
            if (!isfinite(rp->pt_light_dir[a]) || !isfinite(rp->pt_light[a]) || !isfinite(rp->pt_ambient[a]))
                return fail(CINR_INVALID_ARG, "non-finite light parameters");
        if ((int64_t)cam->width * cam->height >= kMaxPathPixels)
            return fail(CINR_INVALID_ARG, "width*height >= 2^27 for the path tracer");
        if (rp->ert_record) return fail(CINR_INVALID_ARG, "ert_record is a ray-marching output");
        if (rp->mode == CINR_UNCACHED_LATTICE) return fail(CINR_INVALID_ARG, "the lattice mode is ray-marching only");
    }
    if (rp->mode == CINR_UNCACHED_LATTICE && rp->samples_per_iter < 8)
        return fail(CINR_INVALID_ARG, "the lattice mode needs samples_per_iter >= 8");
    const bool cached = rp->mode == CINR_CACHED;
    if (cached && !c) return fail(CINR_INVALID_ARG, "the cached mode needs a cache");
    const int vi = cached ? c->index_of(v) : -1;
    if (cached && vi < 0) return fail(CINR_INVALID_ARG, "the volume is not one of the cache's volumes");
    if (cached && rp->frame_index < 0) return fail(CINR_INVALID_ARG, "frame_index must be >= 0");
    st = check_shape(v, rp->mlp_dtype);
    if (st) return st;
    const int64_t npix = (int64_t)cam->width * cam->height;
    const int32_t S = rp->samples_per_iter;
    if (npix * S > 0xFFFFFFFFll) return fail(CINR_INVALID_ARG, "width*height*samples_per_iter >= 2^32");
    const size_t need = render_layout(npix, S, v->n_cells, path, nullptr, nullptr);
    if (!d_ws || ws_bytes < need) return fail(CINR_OUT_OF_MEMORY, "render workspace of %zu bytes < %zu needed", ws_bytes, need);
    // bound on the wavefront iterations: every iteration advances a live ray
    // by >= S samples; a waiting path consumes >= 1 event per iteration
    int64_t max_iters = (int64_t)kPtMaxEvents + 2;
    if (!path) {
        double diag = 0.0;
        for (int a = 0; a < 3; ++a) diag += (double)(v->desc.dims[a] - 1) * (double)(v->desc.dims[a] - 1);
        const double max_samples = ceil(sqrt(diag) / (double)rp->step) + 2.0;
        // the lattice mode gathers S / 8 samples per step (8 values each)
        const int32_t Sg = rp->mode == CINR_UNCACHED_LATTICE ? S / 8 : S;
        max_iters = (int64_t)ceil(max_samples / Sg) + 2;
    }
    if (max_iters > kMaxIters) return fail(CINR_INVALID_ARG, "step too small for samples_per_iter (needs %lld iterations)", (long long)max_iters);
    r.v = v;
    r.npix = npix;
    r.max_iters = max_iters;
    r.queued = npix;
    r.prec = rp->mlp_dtype;
    render_layout(npix, S, v->n_cells, path, &r.L, d_ws);
    const RenderLayout& L = r.L;
    FrameDev& f = r.f;
    f = FrameDev{};
    f.max_iters = (int32_t)max_iters;
    f.view_index = 0;
    f.n_views = 1;
    f.W = cam->width;
    f.H = cam->height;
    f.var = L.var;
    for (int a = 0; a < 3; ++a) {
        f.dims[a] = v->desc.dims[a];
        f.vm1[a] = (float)(v->desc.dims[a] - 1);
        f.M[a] = v->M[a];
    }
    r.hv = frame_var(cached ? c : nullptr, cam, rp);
    f.step = rp->step;
    f.lod_scale = rp->lod_scale;
    f.ert = rp->ert_threshold;
    f.ert_on = rp->ert_threshold <= 1.0f;
    f.ert_rec = rp->ert_record;
    f.S = S;
    f.mode = rp->mode;
    // launch shape: given, or tuned online for this image size
    if (rp->pipe_depth == 0 || rp->xcd_bands == 0) {
        const uint64_t key = ((uint64_t)(uint32_t)cam->width << 32) | (uint32_t)cam->height;
        int cand = 0;
        if (trials) {
            r.tuner = &v->tuners[key];
            cand = r.tuner->cand();
            r.timing_trial = r.tuner->best < 0;
        } else {
            const auto known = v->tuners.find(key);
            if (known != v->tuners.end() && known->second.best >= 0) cand = known->second.best;
        }
        f.pipe = rp->pipe_depth > 0 ? rp->pipe_depth : SamplerTuner::kPipe[cand];
        f.xcd_bands = rp->xcd_bands > 0 ? rp->xcd_bands : SamplerTuner::kBands[cand];
        f.waves = rp->waves_per_simd > 0 ? rp->waves_per_simd : SamplerTuner::kWaves[cand];
        f.claim_rev = SamplerTuner::kRev[cand];
    } else {
        f.pipe = rp->pipe_depth;
        f.xcd_bands = rp->xcd_bands;
        f.waves = rp->waves_per_simd > 0 ? rp->waves_per_simd : 3;
        f.claim_rev = 0;
    }
    f.mc_N = v->desc.macrocell_size;
    f.div_mc = make_fastdiv((uint32_t)(f.mc_N > 0 ? f.mc_N : 1));
    f.flags = v->n_cells > 0 ? L.flags : nullptr;
    f.flag_words = (int32_t)((v->n_cells + 63) / 64);
    // adaptive sampling needs the macro-cells; its codes replace the bits
    f.adapt = v->n_cells > 0 ? rp->adapt_max_exp : 0;
    f.n_cells = v->n_cells;
    f.cell_code = L.cell_code;
    f.vexp = L.vexp;
    if (f.adapt > 0) f.flags = nullptr;
    f.lod_ctx = v->n_cells > 0 ? rp->lod_context : 0.0f;
    f.minmax = v->desc.d_macrocells;
    f.claim = L.claim;
    f.tf = d_tf;
    f.rgba = reinterpret_cast<float4*>(d_rgba);
    if (path) {
        PtDev& pd = f.path;
        pd.on = 1;
        pd.inv_sigma = 1.0f / rp->pt_density;
        for (int a = 0; a < 3; ++a) {
            pd.ldir[a] = rp->pt_light_dir[a];
            pd.light[a] = rp->pt_light[a];
            pd.ambient[a] = rp->pt_ambient[a];
        }
        pd.bounces = rp->pt_max_bounces;
        pd.spp = rp->pt_spp;
        pd.gather = S < kPtGather ? S : kPtGather;
        pd.seed = rp->pt_seed;
        pd.st = L.pts;
    }
    f.k_next = L.k_next;
    f.live0 = L.live0;
    f.live1 = L.live1;
    f.pend_pix = L.pend_pix;
    f.pend_n = L.pend_n;
    // the path tracer's misses are inferred straight into its path state
    f.vals = path ? reinterpret_cast<float*>(L.pts) : L.vals;
    f.miss_rec = L.miss_rec;
    f.ctr = L.ctr;
    f.stats = d_stats ? reinterpret_cast<unsigned long long*>(d_stats) : L.stats;
    if (cached) {
        f.view_table = c->c.views;
        f.geo = c->g;
        f.key_base = (int32_t)(vi * c->g.keys_per_vol);
        f.pt = c->c.pt ? c->c.pt + f.key_base : nullptr;
        f.vdir = c->c.vdir ? c->c.vdir + (int64_t)vi * c->g.dir_per_vol : nullptr;
        f.vblk = c->c.vblk;
        f.last_used = c->c.last_used;
        f.req = c->c.req;
        f.touched = c->c.touched;
        f.n_touched = &c->c.ctr->n_touched;
        f.pool = c->c.pool;
        f.pool16 = c->c.pool16;
        f.pool_kind = c->c.pool_kind;
        f.split = c->c.split;
        f.pool_bricks = c->c.pool_bricks;
        f.misslog = c->c.misslog;
        f.n_misslog = &c->c.ctr->n_misslog;
        f.misslog_cap = c->c.misslog_cap;
    } else {
        f.geo.n_lods = 1;
        f.geo.brick = 2;
    }
    return CINR_OK;
}

cinr_status ensure_readback(cinr_volume v) {
    if (!v->pinned) {
        HIP_TRY(hipHostMalloc((void**)&v->pinned, sizeof(uint32_t) * kMaxViews, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&v->stage, sizeof(FrameVar) * kMaxViews, hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&v->ev, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&v->ev_nf, hipEventDisableTiming | hipEventDisableSystemFence));
    }
    return CINR_OK;
}

// Frame start of a view: counters and macro-cell flags.  `first` also clears
// the frame-wide cache counters (miss log, previous request counts).
cinr_status view_setup(cinr_cache c, ViewRun& r, bool first, hipStream_t s) {
    cinr_volume v = r.v;
    const bool cached = r.f.mode == CINR_CACHED;
    CacheCtr* cctr = cached && first ? c->c.ctr : nullptr;
    const int32_t n_ctr = (int32_t)std::min<int64_t>(r.max_iters + 2, kMaxIters + 2);
    // the host block is read by this frame's k_frame_begin; every frame call
    // waits for its first marches before returning, so the block is free again
    *r.stage = r.hv;
    r.f.var_src = r.stage;
    StageTimer st_(v->timing, s, CINR_STAGE_SETUP);
    HIP_TRY(launch_frame_begin(r.f, n_ctr, v->desc.d_macrocells, v->n_cells, cctr, s));
    if (cached && first && c->c.last_req) HIP_TRY(launch_clear_last_req(c->c, c->g.n_keys, s));
    return CINR_OK;
}

// First march of a view (timed when its launch shape is being tuned).
cinr_status view_march0(ViewRun& r, hipStream_t s) {
    cinr_volume v = r.v;
    SamplerTuner* t = r.tuner;
    if (r.timing_trial) {
        if (!t->a) {
            HIP_TRY(hipEventCreateWithFlags(&t->a, hipEventDisableSystemFence));
            HIP_TRY(hipEventCreateWithFlags(&t->b, hipEventDisableSystemFence));
        }
        HIP_TRY(hipEventRecord(t->a, s));
    }
    {
        StageTimer st_(v->timing, s, CINR_STAGE_MARCH);
        HIP_TRY(launch_march(r.f, 0, r.queued, s));
    }
    if (r.timing_trial) {
        HIP_TRY(hipEventRecord(t->b, s));
        t->pending = true;
    }
    r.n_iters = 1;
    return CINR_OK;
}

// After the pending count of iteration it is known: stop, or infer the misses,
// composite the gathered steps and march the next iteration.
cinr_status view_continue(ViewRun& r, uint32_t pending, Timing& tm, hipStream_t s) {
    const int it = r.n_iters - 1;
    r.queued = pending;
    if (pending == 0 || r.n_iters >= r.max_iters) {
        r.live = false;
        return CINR_OK;
    }
    cinr_volume v = r.v;
    {
        StageTimer st_(tm, s, CINR_STAGE_INFER);
        HIP_TRY(inr_infer_misses(v->m, r.f.miss_rec, &r.f.ctr[it].misses, r.npix * r.f.S, r.f.vals, r.prec, s));
    }
    {
        StageTimer st_(tm, s, CINR_STAGE_SHADE);
        HIP_TRY(launch_shade(r.f, it, r.npix, s));
    }
    {
        StageTimer st_(tm, s, CINR_STAGE_MARCH);
        HIP_TRY(launch_march(r.f, it + 1, r.queued, s));
    }
    r.n_iters += 1;
    return CINR_OK;
}

// Wavefront iteration `it` >= 1 of a view queued without knowing how many
// rays the previous one left: the launches read their counts on the device
// (nothing to do when no ray is pending) and the march takes its full
// persistent grid.
cinr_status view_device_iteration(ViewRun& r, int it, hipStream_t s) {
    HIP_TRY(inr_infer_misses(r.v->m, r.f.miss_rec, &r.f.ctr[it - 1].misses, r.npix * r.f.S, r.f.vals, r.prec, s));
    HIP_TRY(launch_shade(r.f, it - 1, r.npix, s));
    HIP_TRY(launch_march(r.f, it, r.npix, s));
    return CINR_OK;
}

// Tuner bookkeeping once the view's first march has completed.
cinr_status tuner_collect(ViewRun& r, uint32_t first_pending) {
    SamplerTuner* t = r.tuner;
    if (!r.timing_trial || !t || !t->pending) return CINR_OK;
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, t->a, t->b));
    t->pending = false;
    // frames under a pre-load LoD floor sample coarse, coherent bricks and
    // cost far less per sample than the frames that follow: not counted
    if (r.hv.lod_floor > 0) return CINR_OK;
    if (first_pending != 0u && t->waited < SamplerTuner::kMaxWait) {
        t->waited += 1;  // the same candidate is tried again on the next frame
        return CINR_OK;
    }
    // time per sample: consecutive frames of an orbit differ in work by more
    // than the candidates differ in speed.  The first march's samples are
    // committed before it hands its pending count over, and nothing later in
    // the frame changes them.
    unsigned long long n = 0ull;
    HIP_TRY(hipMemcpyAsync(&n, &r.f.stats[ST_SAMPLES], sizeof n, hipMemcpyDeviceToHost, r.st));
    HIP_TRY(hipStreamSynchronize(r.st));
    t->ms[SamplerTuner::of_trial(t->trial)] += n ? ms * 1e6f / (float)n : ms;
    t->trial += 1;
    if (t->trial >= SamplerTuner::kCand * SamplerTuner::kRounds) {
        int best = 0;
        for (int i = 1; i < SamplerTuner::kCand; ++i)
            if (t->ms[i] < t->ms[best]) best = i;
        t->best = best;
    }
    return CINR_OK;
}

cinr_status ensure_side_streams(cinr_cache c) {
    if (c->fork) return CINR_OK;
    for (int k = 0; k < cinr_cache_s::kViewStreams; ++k) {
        HIP_TRY(hipStreamCreateWithFlags(&c->vs[k], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&c->join[k], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    return CINR_OK;
}

// Joins the side streams of a multi-view frame back into `s`.
cinr_status join_side_streams(cinr_cache c, hipStream_t s) {
    for (int k = 0; k < cinr_cache_s::kViewStreams; ++k) {
        HIP_TRY(hipEventRecord(c->join[k], c->vs[k]));
        HIP_TRY(hipStreamWaitEvent(s, c->join[k], 0));
    }
    return CINR_OK;
}

// Frame start of all views: set-up and first march of each, on the view's
// stream (runs[i].st).  With `side`, the views' streams are forked from `s`
// after the first view's set-up, which clears the frame-wide counters.
cinr_status start_views(cinr_cache c, std::vector<ViewRun>& runs, bool side, hipStream_t s) {
    cinr_status st = view_setup(c, runs[0], true, s);
    if (st) return st;
    if (side) {
        HIP_TRY(hipEventRecord(c->fork, s));
        for (int k = 0; k < cinr_cache_s::kViewStreams; ++k) HIP_TRY(hipStreamWaitEvent(c->vs[k], c->fork, 0));
    }
    for (size_t i = 0; i < runs.size(); ++i) {
        if (i > 0) {
            st = view_setup(c, runs[i], false, runs[i].st);
            if (st) return st;
        }
        st = view_march0(runs[i], runs[i].st);
        if (st) return st;
    }
    return CINR_OK;
}

// Wavefront iterations after the first march, to completion; the pending
// counts of all live views are read back with one synchronisation per round
// (into `pinned`).  `known`, when given, holds the counts of the first round,
// already on the host.  With `side`, the view streams are joined into `s` at
// the end, so that everything of the views precedes the cache manager.
cinr_status continue_views(cinr_cache c, std::vector<ViewRun>& runs, bool side, uint32_t* pinned, hipEvent_t ev,
                           const uint32_t* known, hipStream_t s) {
    for (bool have = known != nullptr;; have = false) {
        if (!have) {
            int n_live = 0;
            for (size_t i = 0; i < runs.size(); ++i) {
                if (!runs[i].live) continue;
                const int it = runs[i].n_iters - 1;
                HIP_TRY(hipMemcpyAsync(pinned + i, &runs[i].f.ctr[it].pending, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                       runs[i].st));
                ++n_live;
            }
            if (n_live == 0) break;
            if (side) {
                for (int k = 0; k < cinr_cache_s::kViewStreams; ++k) HIP_TRY(hipEventRecord(c->join[k], c->vs[k]));
                for (int k = 0; k < cinr_cache_s::kViewStreams; ++k) HIP_TRY(hipEventSynchronize(c->join[k]));
            } else {
                HIP_TRY(hipEventRecord(ev, s));
                HIP_TRY(hipEventSynchronize(ev));
            }
        }
        for (size_t i = 0; i < runs.size(); ++i) {
            if (!runs[i].live) continue;
            const uint32_t pending = have ? known[i] : ((volatile uint32_t*)pinned)[i];
            cinr_status st = tuner_collect(runs[i], pending);
            if (st) return st;
            st = view_continue(runs[i], pending, runs[i].v->timing, runs[i].st);
            if (st) return st;
        }
    }
    if (side) return join_side_streams(c, s);
    return CINR_OK;
}

// Whether the next cache-manager pass may need LRU victims (host bound on the
// occupied slots).
bool lru_pass_needed(cinr_cache c) {
    const int64_t p0 = c->c.split, p1 = c->c.pool_bricks - c->c.split;
    return (p0 > 0 && c->used_bound[0] + c->lim > p0) || (p1 > 0 && c->used_bound[1] + c->lim > p1);
}

void note_insertions(cinr_cache c) { note_fill(c, c->lim); }

cinr_status cache_end_frame(cinr_cache c, int32_t prec, bool lru_pass, Timing& tm, const uint32_t* gate, hipStream_t s);

// Frame end of the views: cache manager and decoding (cached frames, c set;
// the selection launch also writes every view's statistics) or each view's
// statistics (uncached); nothing runs unless *gate != 0 when a gate is given.
cinr_status end_views(cinr_cache c, std::vector<ViewRun>& runs, bool lru_pass, Timing& tm, const uint32_t* gate,
                      hipStream_t s) {
    if (c) return cache_end_frame(c, runs[0].prec, lru_pass, tm, gate, s);
    const size_t n = runs.size();
    for (size_t i = 0; i < n; ++i)
        HIP_TRY(launch_frame_end(runs[i].f, (int)runs[i].max_iters, nullptr, i + 1 == n, gate, s));
    return CINR_OK;
}

// One frame of the views `runs` (through cache c when it is cached), to
// completion.  The first marches of all views are followed by one launch that
// copies their pending-ray counts to the host and sets the frame-end gate
// (no ray pending); the frame end is queued right behind it, gated, so that
// the GPU does not wait for the host between the marches and the cache
// manager.  When a view has rays pending (true misses), the gated end does
// nothing: the remaining iterations run, then the end is launched again
// without the gate.  Several views of a cached frame run on the cache's side
// streams so that their marches overlap.
// Value of the pinned pending-count word before the first march stores it.
constexpr uint32_t kPendingUnset = 0xFFFFFFFFu;

// Marks the n pending-count words as not yet stored.  No GPU work of an
// earlier frame writes them any more: the host read them before that frame's
// call returned.
static void reset_pending(uint32_t* pinned, int n) {
    for (int i = 0; i < n; ++i) ((volatile uint32_t*)pinned)[i] = kPendingUnset;
}

// Waits for the n pending counts that the first marches hand over (stored
// after a system-scope fence into pinned host memory, by the last workgroup
// of a single view's march or by k_pending_gather).  Polling the words
// returns as soon as they land; a blocking event wait over a whole march
// tends to sleep and wake late.  The event, recorded after the hand-over, is
// queried every few thousand polls, so that a failed launch ends the wait
// with its error.
static cinr_status poll_pending(const uint32_t* pinned, int n, hipEvent_t ev) {
    const volatile uint32_t* w = pinned;
    auto stored = [&]() {
        for (int i = 0; i < n; ++i)
            if (w[i] == kPendingUnset) return false;
        return true;
    };
    for (uint32_t spin = 1;; ++spin) {
        if (stored()) return CINR_OK;
        __builtin_ia32_pause();  // a spin-wait hint to the core
        if ((spin & 4095u) == 0u) {
            const hipError_t e = hipEventQuery(ev);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return fail(CINR_HIP_ERROR, "frame: %s", hipGetErrorString(e));
            if (stored()) return CINR_OK;
            return fail(CINR_BAD_STATE, "the first marches finished without storing their pending counts");
        }
    }
}

cinr_status render_frame_views(cinr_cache c, std::vector<ViewRun>& runs, Timing& tm, hipStream_t s) {
    cinr_volume rv = runs[0].v;
    cinr_status st = ensure_readback(rv);
    if (st) return st;
    const bool side = c && runs.size() > 1;
    if (side) {
        st = ensure_side_streams(c);
        if (st) return st;
    }
    for (size_t i = 0; i < runs.size(); ++i) {
        runs[i].st = side ? c->vs[i % cinr_cache_s::kViewStreams] : s;
        runs[i].stage = rv->stage + i;
    }
    uint32_t* gate = runs[0].L.gate;
    uint32_t* pinned = (uint32_t*)rv->pinned;
    // one ray-marched view: its first march hands over the pending count
    const bool fused = runs.size() == 1 && !runs[0].f.path.on;
    reset_pending(pinned, (int)runs.size());
    if (fused) {
        runs[0].f.gather_host = pinned;
        runs[0].f.gather_gate = gate;
        runs[0].f.exit_ticket = runs[0].L.ticket;
    }
    st = start_views(c, runs, side, s);
    if (fused) runs[0].f.gather_host = runs[0].f.gather_gate = runs[0].f.exit_ticket = nullptr;
    if (st) return st;
    if (side) {
        st = join_side_streams(c, s);
        if (st) return st;
    }
    std::vector<const FrameDev*> fs;
    for (const ViewRun& r : runs) fs.push_back(&r.f);
    if (!fused) HIP_TRY(launch_pending_gather(fs.data(), (int)runs.size(), 0, pinned, gate, s));
    HIP_TRY(hipEventRecord(rv->ev_nf, s));
    const bool lru = c && lru_pass_needed(c);
    st = end_views(c, runs, lru, tm, gate, s);
    if (st) return st;
    bool trial = false;
    for (const ViewRun& r : runs) trial = trial || (r.timing_trial && r.tuner && r.tuner->pending);
    if (!trial) {
        st = poll_pending(pinned, (int)runs.size(), rv->ev_nf);
        if (st) return st;
    } else {
        // a launch-shape trial's end event must have completed before it is
        // timed
        HIP_TRY(hipEventSynchronize(rv->ev_nf));
    }
    std::vector<uint32_t> known(runs.size());
    bool tail = false;
    for (size_t i = 0; i < runs.size(); ++i) {
        known[i] = ((volatile uint32_t*)pinned)[i];
        tail = tail || known[i] != 0u;
    }
    if (tail) {
        if (side) {
            HIP_TRY(hipEventRecord(c->fork, s));
            for (int k = 0; k < cinr_cache_s::kViewStreams; ++k) HIP_TRY(hipStreamWaitEvent(c->vs[k], c->fork, 0));
        }
        st = continue_views(c, runs, side, pinned, rv->ev, known.data(), s);
        if (st) return st;
        st = end_views(c, runs, lru, tm, nullptr, s);
        if (st) return st;
    } else {
        for (ViewRun& r : runs) {
            st = tuner_collect(r, 0u);
            if (st) return st;
        }
    }
    if (c) note_insertions(c);
    return CINR_OK;
}

// End of a cached frame: ranking and selection of the requests of all views,
// insertion (free slots, then LRU victims), the views' statistics and
// decoding of the new bricks.  Without an LRU pass, ranking, selection,
// insertion and statistics are one launch (when the selection takes two
// passes, its last workgroup runs the second).
cinr_status cache_end_frame(cinr_cache c, int32_t prec, bool lru_pass, Timing& tm, const uint32_t* gate, hipStream_t s) {
    const CacheDev& cd = c->c;
    {
        StageTimer st_(tm, s, CINR_STAGE_CM);
        // ranking of the requested bricks fused into the first selection pass;
        // the request list is published by the last pass
        TopkArgs ta{};
        ta.in = cd.cand;
        ta.count_dev = &cd.ctr->n_touched;
        ta.cap0 = (uint64_t)c->g.n_keys;
        ta.k = c->lim;
        ta.mode = TOPK_RANK;
        ta.frame_gate = gate;
        ta.ra = RankArgs{cd.touched, cd.req, cd.last_req, cd.rank, &cd.ctr->frame, cd.rank_window, cd.ranking};
        SelectArgs sel{cd.ins_keys, cd.ctr, cd.pool_bricks, c->lim};
        ta.tail.insert = lru_pass ? 0 : 1;
        ta.tail.stats = 1;
        ta.tail.c = cd;
        ta.tail.g = c->g;
        uint32_t* fuse = c->plan_sel.n_pass >= 2 ? &cd.ctr->select_done : nullptr;
        HIP_TRY(launch_topk(ta, c->plan_sel, cd.topk[0], cd.topk[1], cd.sel, &sel, fuse, s));
        // LRU victims, only when the pool may be full (the pass is also gated
        // on the device by the number of slots to evict)
        if (lru_pass) {
            TopkArgs tv{};
            tv.count_dev = &cd.ctr->n_used;
            tv.cap0 = (uint64_t)cd.split;
            tv.k = c->lim;
            tv.gate = &cd.ctr->need_evict;
            tv.mode = TOPK_LRU;
            tv.frame_gate = gate;
            tv.lru_last_used = cd.last_used;
            HIP_TRY(launch_topk(tv, c->plan_vic, cd.topk[0], cd.topk[1], cd.vic, nullptr, nullptr, s));
            if (cd.pool_kind == POOL_MIXED) {
                // the binary16 class's own LRU order
                tv.count_dev = &cd.ctr->n_used1;
                tv.cap0 = (uint64_t)(cd.pool_bricks - cd.split);
                tv.gate = &cd.ctr->need_evict1;
                tv.lru_base = cd.split;
                HIP_TRY(launch_topk(tv, c->plan_vic, cd.topk[0], cd.topk[1], cd.vic1, nullptr, nullptr, s));
            }
            HIP_TRY(launch_insert(cd, c->g, c->lim, gate, s));
        }
        if (cd.vdir) HIP_TRY(launch_vpt_update(cd, c->g, gate, s));
    }
    {
        StageTimer st_(tm, s, CINR_STAGE_DECODE);
        HIP_TRY(decode_selected(c, c->lim, prec, gate, s));
    }
    return CINR_OK;
}

}  // namespace

extern "C" cinr_status cinr_render_frame(cinr_cache c, cinr_volume v, const cinr_camera* cam, const float* d_tf,
                                         const cinr_render_params* rp, float* d_rgba, cinr_frame_stats* d_stats,
                                         void* d_ws, size_t ws_bytes, void* stream) {
    std::vector<ViewRun> runs(1);
    cinr_status st = prepare_view(c, v, cam, d_tf, rp, d_rgba, d_stats, d_ws, ws_bytes, runs[0]);
    if (st) return st;
    return render_frame_views(rp->mode == CINR_CACHED ? c : nullptr, runs, v->timing, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Frames without allocation
// ---------------------------------------------------------------------------

// Fixed device array behind cinr_render_frame_noalloc.  Each device holds its
// own copy at its own address; host code takes that address from
// hipGetSymbolAddress (once per device) and never uses the name itself as a
// device pointer.
static __device__ __align__(256) unsigned char scratch[CINR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
// the render workspace, then 256 bytes of control words (the pending-count
// hand-over of the first march)
constexpr size_t kNoAllocWs = CINR_NOALLOC_SCRATCH_BYTES - 256;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of the fixed array on the current device.
cinr_status noalloc_scratch(unsigned char** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CINR_UNSUPPORTED, "device %d (at most %d devices)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(CINR_HIP_ERROR, "the fixed scratch array has no device address");
        g_scratch[dev] = (unsigned char*)p;
    }
    *out = g_scratch[dev];
    return CINR_OK;
}

// A device word on the host, in stream order (the copy goes to pageable
// memory; the stream is synchronised).
cinr_status read_word(const uint32_t* d, uint32_t* h, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(h, d, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return CINR_OK;
}

}  // namespace

extern "C" cinr_status cinr_render_frame_noalloc(cinr_cache c, cinr_volume v, const cinr_camera* cam,
                                                 const float* d_tf, const cinr_render_params* rp, float* d_rgba,
                                                 cinr_frame_stats* d_stats, void* stream) {
    if (!v || !cam || !rp) return fail(CINR_INVALID_ARG, "null argument");
    if (cam->width < 1 || cam->height < 1) return fail(CINR_INVALID_ARG, "empty image");
    if (rp->samples_per_iter < 1 || rp->samples_per_iter > 64)
        return fail(CINR_INVALID_ARG, "samples_per_iter must be in [1, 64]");
    const int64_t npix = (int64_t)cam->width * cam->height;
    if (npix * rp->samples_per_iter > 0xFFFFFFFFll)
        return fail(CINR_INVALID_ARG, "width*height*samples_per_iter >= 2^32");
    const size_t need = render_layout(npix, rp->samples_per_iter, v->n_cells, rp->pipeline == CINR_PATH_TRACE,
                                      nullptr, nullptr);
    if (need > kNoAllocWs)
        return fail(CINR_OUT_OF_MEMORY, "the frame needs %zu bytes of workspace; the fixed scratch array holds %zu "
                    "(reduce width*height or samples_per_iter)", need, kNoAllocWs);
    unsigned char* base = nullptr;
    cinr_status st = noalloc_scratch(&base);
    if (st) return st;
    ViewRun r;
    st = prepare_view(c, v, cam, d_tf, rp, d_rgba, d_stats, base, kNoAllocWs, r, false);
    if (st) return st;
    cinr_cache cc = rp->mode == CINR_CACHED ? c : nullptr;
    hipStream_t s = (hipStream_t)stream;
    uint32_t* word = reinterpret_cast<uint32_t*>(base + kNoAllocWs);
    Timing none;
    r.st = s;
    // frame values from the launch arguments instead of a pinned block
    HIP_TRY(launch_store_var(r.hv, r.L.var, s));
    r.f.var_src = nullptr;
    // a ray-marched view's first march hands its pending count over to the
    // control word and the frame-end gate; the path tracer's goes through
    // the gather launch
    const bool fused = !r.f.path.on;
    if (fused) {
        r.f.gather_host = word;
        r.f.gather_gate = r.L.gate;
        r.f.exit_ticket = r.L.ticket;
    }
    const int32_t n_ctr = (int32_t)std::min<int64_t>(r.max_iters + 2, kMaxIters + 2);
    HIP_TRY(launch_frame_begin(r.f, n_ctr, v->desc.d_macrocells, v->n_cells, cc ? cc->c.ctr : nullptr, s));
    if (cc && cc->c.last_req) HIP_TRY(launch_clear_last_req(cc->c, cc->g.n_keys, s));
    HIP_TRY(launch_march(r.f, 0, r.queued, s));
    r.n_iters = 1;
    if (fused) {
        r.f.gather_host = r.f.gather_gate = r.f.exit_ticket = nullptr;
    } else {
        const FrameDev* fp = &r.f;
        HIP_TRY(launch_pending_gather(&fp, 1, 0, word, r.L.gate, s));
    }
    // the frame end, gated on the device (nothing runs while rays pend)
    const bool lru = cc && lru_pass_needed(cc);
    auto frame_end = [&](const uint32_t* gate) -> cinr_status {
        if (cc) return cache_end_frame(cc, r.prec, lru, none, gate, s);
        HIP_TRY(launch_frame_end(r.f, (int)r.max_iters, nullptr, true, gate, s));
        return CINR_OK;
    };
    st = frame_end(r.L.gate);
    if (st) return st;
    uint32_t pending = 0;
    st = read_word(word, &pending, s);
    if (st) return st;
    if (pending != 0u) {
        // true misses: the remaining iterations, then the frame end
        for (;;) {
            st = view_continue(r, pending, none, s);
            if (st) return st;
            if (!r.live) break;
            st = read_word(&r.f.ctr[r.n_iters - 1].pending, &pending, s);
            if (st) return st;
        }
        st = frame_end(nullptr);
        if (st) return st;
    }
    if (cc) note_insertions(cc);
    return CINR_OK;
}

namespace {

// Validation and descriptors of the views of one multi-view frame.
cinr_status prepare_views(cinr_cache c, int32_t n_views, const cinr_view* views, std::vector<ViewRun>& runs) {
    if (!c || !views) return fail(CINR_INVALID_ARG, "null argument");
    if (n_views < 1 || n_views > kMaxViews) return fail(CINR_INVALID_ARG, "%d views (1 to %d)", n_views, kMaxViews);
    runs.assign(n_views, ViewRun{});
    for (int i = 0; i < n_views; ++i) {
        const cinr_view& w = views[i];
        if (w.params.mode != CINR_CACHED) return fail(CINR_INVALID_ARG, "view %d: views render in the cached mode", i);
        if (w.params.frame_index != views[0].params.frame_index || w.params.mlp_dtype != views[0].params.mlp_dtype)
            return fail(CINR_INVALID_ARG, "view %d: frame_index and mlp_dtype must equal those of view 0", i);
        for (int j = 0; j < i; ++j)
            if (views[j].d_workspace == w.d_workspace) return fail(CINR_INVALID_ARG, "views %d and %d share a workspace", j, i);
        cinr_status st = prepare_view(c, w.volume, &w.camera, w.d_tf, &w.params, w.d_rgba, w.d_stats, w.d_workspace,
                                      w.workspace_bytes, runs[i]);
        if (st) return fail(st, "view %d: %s", i, cinr_last_error());
        // views march concurrently on side streams: the 4-wave register
        // budget lets the views' waves share the CUs (the tuner times each
        // view alone, which favours 3); a caller's choice is kept
        if (n_views > 1 && w.params.waves_per_simd == 0) runs[i].f.waves = 4;
        runs[i].f.view_index = i;
        runs[i].f.n_views = n_views;
    }
    return CINR_OK;
}

}  // namespace

extern "C" cinr_status cinr_render_views(cinr_cache c, int32_t n_views, const cinr_view* views, void* stream) {
    std::vector<ViewRun> runs;
    cinr_status st = prepare_views(c, n_views, views, runs);
    if (st) return st;
    return render_frame_views(c, runs, views[0].volume->timing, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Captured multi-view frames
// ---------------------------------------------------------------------------

constexpr int32_t kMaxDeviceIters = 16;

struct cinr_frame_graph_s {
    cinr_cache c = nullptr;
    std::vector<cinr_view> views;
    FrameVar* stage = nullptr;    // pinned [n]: per-frame values, read by the captured k_frame_begin launches
    uint32_t* pending = nullptr;  // pinned [n]: rays pending after the first marches, written by the start graph
    hipStream_t cs = nullptr;     // capture stream (default priority)
    hipEvent_t ev = nullptr;
    // the whole frame: set-up and first march of every view, pending counts,
    // then cache manager, decoding and frame ends gated on no pending ray;
    // [1] with the LRU victim pass
    hipGraphExec_t frame[2] = {nullptr, nullptr};
    int32_t dev_iters = 0;  // wavefront iterations after the first march queued in the graph
    int64_t n_graph = 0, n_eager = 0, n_tail = 0;
    ~cinr_frame_graph_s() {
        for (hipGraphExec_t e : frame)
            if (e) (void)hipGraphExecDestroy(e);
        if (ev) (void)hipEventDestroy(ev);
        if (cs) (void)hipStreamDestroy(cs);
        if (stage) (void)hipHostFree(stage);
        if (pending) (void)hipHostFree(pending);
    }
};

namespace {

// Switches stage timing off for the volumes of a frame while it is captured
// (timing events are not part of a graph).
struct TimingOff {
    std::vector<std::pair<cinr_volume, bool>> saved;
    explicit TimingOff(const std::vector<ViewRun>& runs) {
        for (const ViewRun& r : runs) {
            saved.emplace_back(r.v, r.v->timing.on);
            r.v->timing.on = false;
        }
    }
    ~TimingOff() {
        for (auto it = saved.rbegin(); it != saved.rend(); ++it) it->first->timing.on = it->second;
    }
};

// Captures `body(stream)` on the graph's capture stream into *exec.
template <class Body>
cinr_status capture(cinr_frame_graph g, hipGraphExec_t* exec, Body body) {
    HIP_TRY(hipStreamBeginCapture(g->cs, hipStreamCaptureModeRelaxed));
    const cinr_status st = body(g->cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(g->cs, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(CINR_HIP_ERROR, "graph capture: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return fail(CINR_HIP_ERROR, "graph instantiation: %s", hipGetErrorString(e2));
    return CINR_OK;
}

}  // namespace

extern "C" cinr_status cinr_frame_graph_create(cinr_cache c, int32_t n_views, const cinr_view* views,
                                               cinr_frame_graph* out) {
    if (!out) return fail(CINR_INVALID_ARG, "null argument");
    *out = nullptr;
    std::vector<ViewRun> runs;
    cinr_status st = prepare_views(c, n_views, views, runs);
    if (st) return st;
    st = ensure_readback(runs[0].v);
    if (st) return st;
    if (n_views > 1) {
        st = ensure_side_streams(c);
        if (st) return st;
    }
    std::unique_ptr<cinr_frame_graph_s> g(new cinr_frame_graph_s);
    g->c = c;
    g->views.assign(views, views + n_views);
    HIP_TRY(hipHostMalloc((void**)&g->stage, sizeof(FrameVar) * n_views, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void**)&g->pending, sizeof(uint32_t) * n_views, hipHostMallocDefault));
    HIP_TRY(hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g->ev, hipEventDisableTiming | hipEventDisableSystemFence));
    *out = g.release();
    return CINR_OK;
}

extern "C" void cinr_frame_graph_destroy(cinr_frame_graph g) { delete g; }

extern "C" cinr_status cinr_frame_graph_render(cinr_frame_graph g, const cinr_camera* cameras, int32_t frame_index,
                                               void* stream) {
    if (!g || !cameras) return fail(CINR_INVALID_ARG, "null argument");
    const int32_t n = (int32_t)g->views.size();
    std::vector<cinr_view> vw = g->views;
    for (int32_t i = 0; i < n; ++i) {
        const cinr_camera& a = cameras[i];
        const cinr_camera& b = g->views[i].camera;
        if (a.width != b.width || a.height != b.height || a.projection != b.projection)
            return fail(CINR_INVALID_ARG, "view %d: the camera's size and projection must stay those the graph was made with", i);
        vw[i].camera = a;
        vw[i].params.frame_index = frame_index;
    }
    cinr_cache c = g->c;
    std::vector<ViewRun> runs;
    cinr_status st = prepare_views(c, n, vw.data(), runs);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    // launch shapes still being tuned online: eager frames
    bool tuned = true;
    for (const ViewRun& r : runs) tuned = tuned && !r.timing_trial;
    if (!tuned) {
        g->n_eager += 1;
        return render_frame_views(c, runs, runs[0].v->timing, s);
    }
    const bool side = n > 1;
    for (int32_t i = 0; i < n; ++i) {
        runs[i].st = side ? c->vs[i % cinr_cache_s::kViewStreams] : g->cs;
        runs[i].stage = g->stage + i;
    }
    const bool lru = lru_pass_needed(c);
    // iterations queued on the device: at most every view's bound minus the first
    int32_t K = g->dev_iters;
    for (const ViewRun& r : runs) K = (int32_t)std::min<int64_t>(K, r.max_iters - 1);
    if (K < 0) K = 0;
    // one ray-marched view and no queued iteration: its first march hands
    // the pending count over itself, as in eager frames
    const bool fused = n == 1 && K == 0 && !runs[0].f.path.on;
    if (!g->frame[lru]) {
        TimingOff off(runs);
        Timing none;
        st = capture(g, &g->frame[lru], [&](hipStream_t cs) -> cinr_status {
            if (fused) {
                runs[0].f.gather_host = g->pending;
                runs[0].f.gather_gate = runs[0].L.gate;
                runs[0].f.exit_ticket = runs[0].L.ticket;
            }
            cinr_status r = start_views(c, runs, side, cs);
            if (fused) runs[0].f.gather_host = runs[0].f.gather_gate = runs[0].f.exit_ticket = nullptr;
            if (r) return r;
            if (side) {
                r = join_side_streams(c, cs);
                if (r) return r;
            }
            for (int32_t k = 1; k <= K; ++k)
                for (ViewRun& v : runs) {
                    r = view_device_iteration(v, k, cs);
                    if (r) return r;
                }
            if (!fused) {
                std::vector<const FrameDev*> fs;
                for (const ViewRun& v : runs) fs.push_back(&v.f);
                HIP_TRY(launch_pending_gather(fs.data(), n, K, g->pending, runs[0].L.gate, cs));
            }
            return end_views(c, runs, lru, none, runs[0].L.gate, cs);
        });
        if (st) return st;
    }
    for (int32_t i = 0; i < n; ++i) g->stage[i] = runs[i].hv;
    reset_pending(g->pending, n);
    // one graph per frame; its frame end does nothing if a view still has
    // rays pending after the first marches and the K iterations behind them
    HIP_TRY(hipGraphLaunch(g->frame[lru], s));
    HIP_TRY(hipEventRecord(g->ev, s));
    st = poll_pending(g->pending, n, g->ev);
    if (st) return st;
    std::vector<uint32_t> known(n);
    bool tail = false;
    for (int32_t i = 0; i < n; ++i) {
        known[i] = ((volatile uint32_t*)g->pending)[i];
        runs[i].n_iters = 1 + K;
        runs[i].st = s;
        tail = tail || known[i] != 0u;
    }
    if (tail) {
        // rays left after the queued iterations (true misses): the remaining
        // iterations and the frame end run eagerly on `s`
        g->n_tail += 1;
        cinr_volume rv = runs[0].v;
        st = continue_views(c, runs, false, (uint32_t*)rv->pinned, rv->ev, known.data(), s);
        if (st) return st;
        Timing none;
        st = end_views(c, runs, lru, none, nullptr, s);
        if (st) return st;
    }
    note_insertions(c);
    g->n_graph += 1;
    return CINR_OK;
}

extern "C" cinr_status cinr_frame_graph_set_device_iterations(cinr_frame_graph g, int32_t iterations) {
    if (!g) return fail(CINR_INVALID_ARG, "null argument");
    if (iterations < 0 || iterations > kMaxDeviceIters)
        return fail(CINR_INVALID_ARG, "iterations = %d out of [0, %d]", iterations, kMaxDeviceIters);
    if (iterations == g->dev_iters) return CINR_OK;
    // graphs of the old count are captured again on their next use; none of
    // their launches may still be running when they are destroyed
    HIP_TRY(hipDeviceSynchronize());
    for (hipGraphExec_t& e : g->frame) {
        if (e) HIP_TRY(hipGraphExecDestroy(e));
        e = nullptr;
    }
    g->dev_iters = iterations;
    return CINR_OK;
}

extern "C" cinr_status cinr_frame_graph_counts(cinr_frame_graph g, int64_t* graph_frames, int64_t* eager_frames,
                                               int64_t* tail_frames) {
    if (!g || !graph_frames || !eager_frames || !tail_frames) return fail(CINR_INVALID_ARG, "null argument");
    *graph_frames = g->n_graph;
    *eager_frames = g->n_eager;
    *tail_frames = g->n_tail;
    return CINR_OK;
}

extern "C" cinr_status cinr_tuned_launch(cinr_volume v, int32_t width, int32_t height, int32_t* pipe_depth,
                                         int32_t* xcd_bands, int32_t* waves_per_simd, int32_t* trials_left) {
    if (!v || !pipe_depth || !xcd_bands || !waves_per_simd || !trials_left)
        return fail(CINR_INVALID_ARG, "null argument");
    const uint64_t key = ((uint64_t)(uint32_t)width << 32) | (uint32_t)height;
    auto it = v->tuners.find(key);
    if (it == v->tuners.end()) {
        *pipe_depth = *xcd_bands = *waves_per_simd = 0;
        *trials_left = SamplerTuner::kCand * SamplerTuner::kRounds;
        return CINR_OK;
    }
    const SamplerTuner& t = it->second;
    const int cand = t.cand();
    *pipe_depth = SamplerTuner::kPipe[cand];
    *xcd_bands = SamplerTuner::kBands[cand];
    *waves_per_simd = SamplerTuner::kWaves[cand];
    *trials_left = t.best >= 0 ? 0 : SamplerTuner::kCand * SamplerTuner::kRounds - t.trial;
    return CINR_OK;
}

// ---------------------------------------------------------------------------
// Dumps
// ---------------------------------------------------------------------------

extern "C" cinr_status cinr_cache_dump(cinr_cache c, int32_t kind, void* dst, size_t bytes, size_t* needed, void* stream) {
    if (!c || !needed) return fail(CINR_INVALID_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const CacheDev& cd = c->c;
    CacheCtr h{};
    HIP_TRY(hipMemcpyAsync(&h, cd.ctr, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const void* src = nullptr;
    size_t n = 0;
    const size_t nk = (size_t)c->g.n_keys, P = (size_t)cd.pool_bricks;
    const size_t B3 = (size_t)c->g.brick * c->g.brick * c->g.brick;
    const size_t nd = (size_t)(c->g.dir_per_vol * c->g.n_vols);
    if ((kind == CINR_DUMP_PT_DIRECTORY || kind == CINR_DUMP_PT_BLOCKS || kind == CINR_DUMP_PT_STATE) && !cd.vdir)
        return fail(CINR_BAD_STATE, "the cache has a flat page table (virtual_page_table = 0)");
    if (kind == CINR_DUMP_PT_STATE) {
        *needed = 16;
        if (!dst || bytes < 16) return fail(CINR_OUT_OF_MEMORY, "dump needs 16 bytes");
        int32_t* o = (int32_t*)dst;
        o[0] = cd.vcap;
        o[1] = (int32_t)h.v_free;
        o[2] = (int32_t)h.v_fail;
        o[3] = (int32_t)c->g.dir_per_vol;
        return CINR_OK;
    }
    if (kind == CINR_DUMP_PAGE_TABLE && cd.vdir) {
        // the flat view of the two-level table, resolved on the host
        *needed = nk * 4;
        if (!dst || bytes < nk * 4) return fail(CINR_OUT_OF_MEMORY, "dump needs %zu bytes", nk * 4);
        std::vector<int32_t> dir(nd), blk((size_t)cd.vcap * kVptEntries);
        HIP_TRY(hipMemcpyAsync(dir.data(), cd.vdir, nd * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(blk.data(), cd.vblk, blk.size() * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        int32_t* o = (int32_t*)dst;
        for (size_t k = 0; k < nk; ++k) {
            int64_t d;
            int32_t e;
            vpt_addr(c->g, (int64_t)k, &d, &e);
            const int32_t b = dir[(size_t)d];
            o[k] = b < 0 || b >= cd.vcap ? -1 : blk[(size_t)b * kVptEntries + e];
        }
        return CINR_OK;
    }
    switch (kind) {
        case CINR_DUMP_PAGE_TABLE: src = cd.pt; n = nk * 4; break;
        case CINR_DUMP_PT_DIRECTORY: src = cd.vdir; n = nd * 4; break;
        case CINR_DUMP_PT_BLOCKS: src = cd.vblk; n = (size_t)cd.vcap * kVptEntries * 4; break;
        case CINR_DUMP_SLOT_OWNER: src = cd.owner; n = P * 4; break;
        case CINR_DUMP_LAST_USED: src = cd.last_used; n = P * 4; break;
        case CINR_DUMP_RANK: src = cd.rank; n = nk * 8; break;
        case CINR_DUMP_REQ_COUNT:
            if (!cd.last_req) return fail(CINR_BAD_STATE, "request counts are not kept (keep_request_counts = 0)");
            src = cd.last_req;
            n = nk * 4;
            break;
        case CINR_DUMP_REQUEST_LIST: src = cd.ins_keys; n = (size_t)h.n_sel * 4; break;
        case CINR_DUMP_MISS_LIST:
            if ((int64_t)h.n_misslog > cd.misslog_cap) return fail(CINR_BAD_STATE, "miss log overflow: %u records, capacity %d", h.n_misslog, cd.misslog_cap);
            src = cd.misslog;
            n = (size_t)h.n_misslog * sizeof(MissLogRec);
            break;
        case CINR_DUMP_EVICTION_LOG: {
            const size_t m = std::min<size_t>(h.n_evlog, (size_t)cd.evlog_cap);
            src = cd.evlog;
            n = m * 16;
            break;
        }
        case CINR_DUMP_POOL:
            // binary32 slots [0, split), then binary16 slots [split, P)
            src = cd.pool;
            n = cd.pool_kind == POOL_F16 ? P * B3 * 2 : (size_t)cd.split * B3 * 4 + (P - (size_t)cd.split) * B3 * 2;
            break;
        default: return fail(CINR_INVALID_ARG, "dump kind %d", kind);
    }
    *needed = n;
    if (!dst || bytes < n) return fail(CINR_OUT_OF_MEMORY, "dump needs %zu bytes", n);
    if (n == 0) return CINR_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (kind == CINR_DUMP_MISS_LIST) {
        MissLogRec* r = (MissLogRec*)dst;
        std::sort(r, r + h.n_misslog, [](const MissLogRec& a, const MissLogRec& b) {
            return a.pix != b.pix ? a.pix < b.pix : a.k < b.k;
        });
    }
    return CINR_OK;
}

// ---------------------------------------------------------------------------
// Training (the learned part)
// ---------------------------------------------------------------------------

struct cinr_trainer_s {
    cinr_volume vol;
    cinr_train_desc desc;
    int64_t n_table, n_weights, max_waves;
    float *m_t, *v_t, *g_t, *m_w, *v_w, *g_w, *partial, *u, *target, *loss;
};

namespace {

cinr_status check_train(cinr_volume v, const cinr_train_desc* d) {
    if (!v || !d) return fail(CINR_INVALID_ARG, "null argument");
    if (!train_shape_supported(v->m))
        return fail(CINR_UNSUPPORTED, "no training kernel for %d levels x %d features, hidden width %d",
                    v->m.n_levels, v->m.n_features, v->m.hidden);
    if (d->mlp_dtype != CINR_F32 && d->mlp_dtype != CINR_BF16)
        return fail(CINR_UNSUPPORTED, "training runs its MLP in F32 or BF16 (dtype %d)", d->mlp_dtype);
    if (d->batch < 1 || d->batch > (1ll << 31)) return fail(CINR_INVALID_ARG, "batch = %lld", (long long)d->batch);
    if (!(d->lr > 0.0f) || !(d->beta1 >= 0.0f && d->beta1 < 1.0f) || !(d->beta2 >= 0.0f && d->beta2 < 1.0f) ||
        !(d->eps >= 0.0f))
        return fail(CINR_INVALID_ARG, "Adam needs lr > 0, 0 <= beta < 1, eps >= 0");
    return CINR_OK;
}

int64_t train_waves() {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1) return 1024;
    return 4ll * n_cu;
}

size_t train_layout(const cinr_train_desc* d, int64_t n_table, int64_t nw, int64_t waves, cinr_trainer_s* t,
                    void* base) {
    Carver cv(base);
    cinr_trainer_s x{};
    x.m_t = cv.take<float>(n_table);
    x.v_t = cv.take<float>(n_table);
    x.g_t = cv.take<float>(n_table);
    x.m_w = cv.take<float>(nw);
    x.v_w = cv.take<float>(nw);
    x.g_w = cv.take<float>(nw);
    x.partial = cv.take<float>((size_t)waves * (nw + 1));
    x.u = cv.take<float>((size_t)d->batch * 3);
    x.target = cv.take<float>(d->batch);
    x.loss = cv.take<float>(1);
    if (t) {
        t->m_t = x.m_t;
        t->v_t = x.v_t;
        t->g_t = x.g_t;
        t->m_w = x.m_w;
        t->v_w = x.v_w;
        t->g_w = x.g_w;
        t->partial = x.partial;
        t->u = x.u;
        t->target = x.target;
        t->loss = x.loss;
    }
    return cv.off;
}

cinr_status check_grid(const float* grid, const int32_t* dims) {
    if (!grid) return CINR_OK;
    if (!dims) return fail(CINR_INVALID_ARG, "grid without dimensions");
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > (1 << 24)) return fail(CINR_INVALID_ARG, "grid dims[%d] = %d", a, dims[a]);
    return CINR_OK;
}

}  // namespace

extern "C" cinr_status cinr_train_workspace_size(cinr_volume v, const cinr_train_desc* d, size_t* bytes) {
    cinr_status st = check_train(v, d);
    if (st) return st;
    if (!bytes) return fail(CINR_INVALID_ARG, "null argument");
    const int64_t nt = v->table_entries * v->m.n_features;
    *bytes = train_layout(d, nt, train_n_weights(v->m), train_waves(), nullptr, nullptr);
    return CINR_OK;
}

extern "C" cinr_status cinr_train_create(cinr_volume v, const cinr_train_desc* d, void* d_ws, size_t ws_bytes,
                                         void* stream, cinr_trainer* out) {
    cinr_status st = check_train(v, d);
    if (st) return st;
    if (!out) return fail(CINR_INVALID_ARG, "null argument");
    const int64_t nt = v->table_entries * v->m.n_features, nw = train_n_weights(v->m), waves = train_waves();
    const size_t need = train_layout(d, nt, nw, waves, nullptr, nullptr);
    if (!d_ws || ws_bytes < need) return fail(CINR_OUT_OF_MEMORY, "training workspace of %zu bytes < %zu needed", ws_bytes, need);
    cinr_trainer t = new cinr_trainer_s();
    t->vol = v;
    t->desc = *d;
    t->n_table = nt;
    t->n_weights = nw;
    t->max_waves = waves;
    train_layout(d, nt, nw, waves, t, d_ws);
    hipStream_t s = (hipStream_t)stream;
    // Adam moments and the table gradient start at zero
    hipError_t e = fill_f32(t->m_t, nt, 0.0f, s);
    if (e == hipSuccess) e = fill_f32(t->v_t, nt, 0.0f, s);
    if (e == hipSuccess) e = fill_f32(t->g_t, nt, 0.0f, s);
    if (e == hipSuccess) e = fill_f32(t->m_w, nw, 0.0f, s);
    if (e == hipSuccess) e = fill_f32(t->v_w, nw, 0.0f, s);
    if (e == hipSuccess) e = fill_f32(t->g_w, nw, 0.0f, s);
    if (e != hipSuccess) {
        delete t;
        return fail(CINR_HIP_ERROR, "initialising the trainer: %s", hipGetErrorString(e));
    }
    *out = t;
    return CINR_OK;
}

extern "C" void cinr_train_destroy(cinr_trainer t) { delete t; }

extern "C" cinr_status cinr_train_points(cinr_trainer t, const float* d_grid, const int32_t* grid_dims, int64_t step,
                                         float* d_u, float* d_target, void* stream) {
    if (!t || !d_u || (d_grid && !d_target)) return fail(CINR_INVALID_ARG, "null argument");
    if (step < 0) return fail(CINR_INVALID_ARG, "step < 0");
    cinr_status st = check_grid(d_grid, grid_dims);
    if (st) return st;
    HIP_TRY(train_points(t->desc.seed, step, t->desc.batch, d_grid, grid_dims, d_u, d_target, (hipStream_t)stream));
    return CINR_OK;
}

extern "C" cinr_status cinr_train_gradients(cinr_trainer t, const float* d_u, const float* d_target, int64_t n,
                                            float* d_loss, float* d_g_table, float* d_g_weights, void* stream) {
    if (!t || !d_g_table || !d_g_weights || (n > 0 && (!d_u || !d_target))) return fail(CINR_INVALID_ARG, "null argument");
    if (n < 0 || n > (1ll << 31)) return fail(CINR_INVALID_ARG, "n = %lld", (long long)n);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(fill_f32(d_g_table, t->n_table, 0.0f, s));
    HIP_TRY(train_gradients(t->vol->m, t->desc.mlp_dtype, d_u, d_target, n, n > 0 ? 2.0f / (float)n : 0.0f, d_g_table,
                            d_g_weights, d_loss, t->partial, t->max_waves, s));
    return CINR_OK;
}

extern "C" cinr_status cinr_train_step(cinr_trainer t, const float* d_grid, const int32_t* grid_dims, int64_t step,
                                       float* d_loss, void* stream) {
    if (!t || !d_grid) return fail(CINR_INVALID_ARG, "null argument");
    if (step < 0) return fail(CINR_INVALID_ARG, "step < 0");
    cinr_status st = check_grid(d_grid, grid_dims);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const cinr_train_desc& d = t->desc;
    const int64_t n = d.batch;
    HIP_TRY(train_points(d.seed, step, n, d_grid, grid_dims, t->u, t->target, s));
    // the table gradient is zero here: cleared at creation and by every Adam update
    HIP_TRY(train_gradients(t->vol->m, d.mlp_dtype, t->u, t->target, n, 2.0f / (float)n, t->g_t, t->g_w,
                            d_loss ? d_loss : t->loss, t->partial, t->max_waves, s));
    float* table = const_cast<float*>(t->vol->desc.d_table);
    float* weights = const_cast<float*>(t->vol->desc.d_weights);
    HIP_TRY(adam_update(table, t->m_t, t->v_t, t->g_t, t->n_table, d.lr, d.beta1, d.beta2, d.eps, step + 1, true, s));
    HIP_TRY(adam_update(weights, t->m_w, t->v_w, t->g_w, t->n_weights, d.lr, d.beta1, d.beta2, d.eps, step + 1, false, s));
    return CINR_OK;
}

extern "C" cinr_status cinr_train_set_lr(cinr_trainer t, float lr) {
    if (!t) return fail(CINR_INVALID_ARG, "null argument");
    if (!(lr > 0.0f) || !isfinite(lr)) return fail(CINR_INVALID_ARG, "lr must be > 0");
    t->desc.lr = lr;
    return CINR_OK;
}

extern "C" cinr_status cinr_adam_update(float* d_p, float* d_m, float* d_v, float* d_g, int64_t n, int64_t step,
                                        float lr, float beta1, float beta2, float eps, int32_t clear_grad, void* stream) {
    if (n < 0 || (n > 0 && (!d_p || !d_m || !d_v || !d_g))) return fail(CINR_INVALID_ARG, "null argument");
    if (step < 1) return fail(CINR_INVALID_ARG, "Adam steps count from 1");
    HIP_TRY(adam_update(d_p, d_m, d_v, d_g, n, lr, beta1, beta2, eps, step, clear_grad != 0, (hipStream_t)stream));
    return CINR_OK;
}
