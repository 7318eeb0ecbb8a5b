// Wavefront ray marching through the brick cache (Section 5.1 with the
// sampler of Algorithms 1 and 2 and the fallback of Section 4.3).
//
// One frame is: iterations of { march, infer misses, shade } until no ray has
// a deferred step.  `march` is a persistent kernel: every lane owns one ray at
// a time and composites samples as the cache serves them; lanes whose ray has
// ended are refilled from work units (8x8 pixel tiles in the first iteration,
// runs of 64 re-queued rays later) claimed from per-XCD counters.  At the
// first true miss a ray gathers a wavefront step of S samples (the miss
// included) into a per-ray buffer and appends true-miss records, with one
// atomic per wave for each list.  The INR then infers all misses in one batch
// (Algorithm 1), and `shade` composites the gathered samples in order,
// re-queueing unfinished rays for the next iteration.
#include <type_traits>

#include "frame.h"

namespace cinr {


struct SampleRes {
    int32_t status;
    int32_t slot;
    int32_t req_key;
    float value;
    int32_t e;  // step exponent of the sample's macro-cell (adaptive sampling)
};

// The last page-table lookup of a lane at each LoD (LoD L in way L mod 4),
// kept in LDS: way w of a lane at base[w * kBlock] (consecutive lanes,
// consecutive words).  Residency is constant within a frame, so a repeated
// key (consecutive samples in the same brick) needs no reload, and entries
// stay valid from one ray to the next; a sample that falls back from an
// unmapped LoD to coarser ones finds every level it tries here until the ray
// leaves one of the bricks.  A new key reads the flat page table, or the
// directory entry of its block and then the block's entry (two-level table).
constexpr int kSlotWays = 4;
struct SlotCache {
    int2* base;
    __device__ int32_t lookup(const FrameDev& f, const LodGeom& lg, int32_t key, const int32_t b[3], int32_t lod) {
        int2* e = base + (lod & (kSlotWays - 1)) * kBlock;
        const int2 c = *e;
        if (c.x == key) return c.y;
        int32_t v;
        if (f.vdir) {
            const int32_t blk = f.vdir[vpt_dir(lg, b)];
            v = blk < 0 ? -1 : f.vblk[(int64_t)blk * kVptEntries + vpt_entry(b)];
        } else {
            v = f.pt[key];
        }
        *e = make_int2(key, v);
        return v;
    }
};

// Macro-cell flags, staged in LDS or read from global memory.
struct LdsFlags {
    const uint64_t* w;
    __device__ bool get(uint32_t cell) const { return (w[cell >> 6] >> (cell & 63u)) & 1ull; }
};
struct GlobalFlags {
    const uint64_t* w;
    __device__ bool get(uint32_t cell) const { return (w[cell >> 6] >> (cell & 63u)) & 1ull; }
};
// One-byte macro-cell codes of the adaptive sampler (0xFF: transparent).
struct LdsCodes {
    const uint8_t* c;
    __device__ uint32_t code(uint32_t cell) const { return c[cell]; }
};
struct GlobalCodes {
    const uint8_t* c;
    __device__ uint32_t code(uint32_t cell) const { return c[cell]; }
};

// Per-frame values that the sampler reads for every sample (loaded once per
// launch from the frame's device block).
struct FrameHot {
    float eye[3];
    uint32_t seed;
    int32_t lod_floor;
    int32_t frame;
    int32_t preload;
};

__device__ inline FrameHot load_hot(const FrameVar* v) {
    FrameHot h;
#pragma unroll
    for (int a = 0; a < 3; ++a) h.eye[a] = v->cam.eye[a];
    h.seed = v->frame_seed;
    h.lod_floor = v->lod_floor;
    h.frame = v->frame;
    h.preload = v->preload;
    return h;
}

// Sampler of Algorithm 2 for one position: macro-cell skip, stochastic LoD,
// page-table lookup at that LoD and every coarser one, trilinear fetch.  The
// flag read and the first page-table read are issued together; a skipped
// sample discards the lookup.  kFast (nonzero): bricks of 16^3 (compile-time
// brick offsets) and macro-cells of 16^3 voxels; kFast = 1: a pool of less
// than 4 GiB, addressed by 32-bit byte offsets, kFast = 2: any pool, each
// brick's base in 64 bits.  kAdapt: the cell's code (Flags reads codes)
// gives the sample's step exponent; a transparent cell's samples are skipped.
// kPool: POOL_F32, POOL_F16 (binary16 values, interpolated in FP32), or
// POOL_MIXED (binary32 slots below f.split, binary16 slots from it on).
__device__ inline float pool_value(float x) { return x; }
__device__ inline float pool_value(__half x) { return __half2float(x); }

// The 8 pool values around a sample in a brick stored as T at `base`
// (slot relative to base): c[x + 2y + 4z].
template <int kFast, class T>
__device__ inline void brick_corners(const void* base, int32_t slot, const BrickAddr& a, int32_t B, float c[8]) {
    constexpr int kB = kFast ? 16 : 0;
    const T* br;
    if (kFast == 2) {
        // the brick's base in 64 bits, the sample's offset inside it in 32
        const char* b = reinterpret_cast<const char*>(base) + (uint64_t)(uint32_t)slot * (kB * kB * kB * sizeof(T));
        const uint32_t off = (((uint32_t)a.lj[2] * kB + (uint32_t)a.lj[1]) * kB + (uint32_t)a.lj[0]) * (uint32_t)sizeof(T);
        br = reinterpret_cast<const T*>(b + off);
    } else if (kFast) {
        const uint32_t off = (((uint32_t)slot * (uint32_t)(kB * kB * kB) +
                               ((uint32_t)a.lj[2] * kB + (uint32_t)a.lj[1]) * kB + (uint32_t)a.lj[0])) *
                             (uint32_t)sizeof(T);
        br = reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
    } else {
        br = static_cast<const T*>(base) + (int64_t)slot * (B * B * B) + ((int64_t)a.lj[2] * B + a.lj[1]) * B + a.lj[0];
    }
    const int32_t Bq = kFast ? kB : B;
    const int32_t B2 = Bq * Bq;
    c[0] = pool_value(br[0]);
    c[1] = pool_value(br[1]);
    c[2] = pool_value(br[Bq]);
    c[3] = pool_value(br[Bq + 1]);
    c[4] = pool_value(br[B2]);
    c[5] = pool_value(br[B2 + 1]);
    c[6] = pool_value(br[B2 + Bq]);
    c[7] = pool_value(br[B2 + Bq + 1]);
}

template <int kFast, bool kAdapt, int kPool, class Flags>
__device__ inline SampleRes sample_cache(const FrameDev& f, const FrameHot& h, const LodGeom* lg, const Flags& fl,
                                         const float p[3], SlotCache& sc) {
    constexpr int kB = kFast ? 16 : 0;
    SampleRes s;
    s.slot = -1;
    s.req_key = -1;
    s.value = 0.0f;
    s.e = 0;
    bool live = true;
    float lod_factor = 1.0f;
    if (kAdapt || f.flags) {
        uint32_t ci[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ci[a] = kFast ? (uint32_t)(int32_t)p[a] >> 4 : fast_div((uint32_t)(int32_t)p[a], f.div_mc);
            if (ci[a] > (uint32_t)f.M[a] - 1u) ci[a] = (uint32_t)f.M[a] - 1u;
        }
        const uint32_t cell = (ci[2] * (uint32_t)f.M[1] + ci[1]) * (uint32_t)f.M[0] + ci[0];
        if (f.lod_ctx > 0.0f) {
            // context-aware LoD: 1 - kappa * (value range of the cell)
            const float2 mm = reinterpret_cast<const float2*>(f.minmax)[cell];
            const float range = mm.y - mm.x;
            const float k = f.lod_ctx * range;
            lod_factor = 1.0f - k;
        }
        if constexpr (kAdapt) {
            const uint32_t code = fl.code(cell);
            live = code != 0xFFu;
            s.e = live ? (int32_t)code : f.adapt;
        } else {
            live = fl.get(cell);
        }
    }
    if (f.mode != CINR_CACHED) {
        s.status = live ? S_MISS : S_SKIP;
        return s;
    }
    const int32_t nl = f.geo.n_lods;
    const int32_t L = select_lod(p, h.eye, f.lod_scale, lod_factor, h.seed, h.lod_floor, nl);
    const int32_t B = kFast ? kB : f.geo.brick;
    s.status = S_MISS;
    // the first mapped LoD from L on (keys only), then one fetch from it
    int32_t slot = -1, Ls = L;
    for (int32_t Lp = L; Lp < nl; ++Lp) {
        int32_t b[3];
        const int32_t key = brick_key<kB>(lg[Lp], f.geo.brick, f.geo.div_b1, Lp, p, b);
        if (Lp == L) s.req_key = key;
        const int32_t sl = sc.lookup(f, lg[Lp], key, b, Lp);
        if (!live) {
            s.status = S_SKIP;
            s.req_key = -1;
            return s;
        }
        if (sl >= 0) {
            slot = sl;
            Ls = Lp;
            break;
        }
    }
    if (slot < 0) return s;
    const BrickAddr a = brick_addr<kB>(lg[Ls], f.geo.brick, f.geo.div_b1, Ls, p);
    float c[8];
    if constexpr (kPool == POOL_MIXED) {
        if (slot < f.split)
            brick_corners<kFast, float>(f.pool, slot, a, B, c);
        else
            brick_corners<kFast, __half>(f.pool16, slot - f.split, a, B, c);
    } else {
        brick_corners<kFast, typename std::conditional<kPool == POOL_F16, __half, float>::type>(f.pool, slot, a, B, c);
    }
    const float c000 = c[0], c100 = c[1], c010 = c[2], c110 = c[3];
    const float c001 = c[4], c101 = c[5], c011 = c[6], c111 = c[7];
    const float fx = a.frac[0], fy = a.frac[1], fz = a.frac[2];
    const float x00 = __builtin_fmaf(fx, c100 - c000, c000);
    const float x10 = __builtin_fmaf(fx, c110 - c010, c010);
    const float x01 = __builtin_fmaf(fx, c101 - c001, c001);
    const float x11 = __builtin_fmaf(fx, c111 - c011, c011);
    const float y0 = __builtin_fmaf(fy, x10 - x00, x00);
    const float y1 = __builtin_fmaf(fy, x11 - x01, x01);
    s.value = __builtin_fmaf(fz, y1 - y0, y0);
    s.slot = slot;
    s.status = Ls == L ? S_HIT : S_FALLBACK;
    return s;
}

// Transfer function lookup (linear between rows floor(v*255) and the next),
// opacity correction a' = 1 - (1-a)^step, front-to-back compositing.
__device__ inline void composite(float4& acc, float v, const float4* tfs, float step) {
    const float x = v * 255.0f;
    int32_t i0 = (int32_t)x;
    i0 = i0 > 254 ? 254 : (i0 < 0 ? 0 : i0);
    const float t = x - (float)i0;
    const float4 a = tfs[i0], b = tfs[i0 + 1];
    const float r = __builtin_fmaf(t, b.x - a.x, a.x);
    const float g = __builtin_fmaf(t, b.y - a.y, a.y);
    const float bl = __builtin_fmaf(t, b.z - a.z, a.z);
    float al = __builtin_fmaf(t, b.w - a.w, a.w);
    al = al < 0.0f ? 0.0f : (al > 1.0f ? 1.0f : al);
    // value plane: the hardware exp2/log2 (about 1 ulp) are accurate enough
    const float ac = 1.0f - __builtin_amdgcn_exp2f(step * __builtin_amdgcn_logf(1.0f - al));
    const float w = (1.0f - acc.w) * ac;
    acc.x = __builtin_fmaf(w, r, acc.x);
    acc.y = __builtin_fmaf(w, g, acc.y);
    acc.z = __builtin_fmaf(w, bl, acc.z);
    acc.w += w;
}

// Values of one march launch that only its cold paths read (ray setup,
// wavefront steps, request and miss-log appends).  They are staged in LDS and
// read through a volatile pointer at each use, so that they hold no registers
// across the sample loop.
struct MarchCold {
    CamDev cam;
    float4* rgba;
    int32_t* k_next;
    const int32_t* cur;
    int32_t* pend_pix;
    int32_t* pend_n;
    float* vals;
    float4* miss_rec;
    uint32_t* pending;  // counters of this iteration
    uint32_t* misses;
    MissLogRec* misslog;
    uint32_t* n_misslog;
    int32_t misslog_cap;
    uint32_t* req;      // request counts of this frame's volume (offset by key_base)
    int32_t* touched;
    uint32_t* n_touched;
    int32_t key_base;   // global key of the volume's first brick
    int32_t* ert_rec;   // nullable: early-termination record (FrameDev::ert_rec)
};
using ColdRef = const volatile MarchCold*;

__device__ inline CamDev load_cam(const volatile CamDev& v) {
    CamDev c;
    c.proj = v.proj;
    c.W = v.W;
    c.H = v.H;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.eye[a] = v.eye[a];
        c.fwd[a] = v.fwd[a];
        c.right[a] = v.right[a];
        c.up[a] = v.up[a];
    }
    c.tanx = v.tanx;
    c.tany = v.tany;
    c.ow = v.ow;
    c.oh = v.oh;
    return c;
}

__device__ inline void flush_requests(ColdRef c, int32_t key, uint32_t cnt) {
    if (key < 0 || cnt == 0) return;
    uint32_t* req = c->req;
    const uint32_t old = atomicAdd(&req[key], cnt);
    if (old == 0u) {
        const uint32_t i = atomicAdd(c->n_touched, 1u);
        int32_t* touched = c->touched;
        touched[i] = c->key_base + key;
    }
}

// The request runs (key, cnt) of all 64 lanes together, one atomic per
// distinct key of the wave: neighbouring rays of a tile request the same
// bricks, and the counts of a frame's few hundred requested bricks would
// otherwise meet as thousands of atomics per address.  Every lane calls it.
__device__ inline void wave_flush_requests(ColdRef c, int32_t key, uint32_t cnt) {
    bool pend = key >= 0 && cnt != 0u;
    for (uint64_t todo = __ballot(pend); todo != 0ull; todo = __ballot(pend)) {
        const int leader = __builtin_ctzll(todo);
        const int32_t lk = __shfl(key, leader);
        const bool same = pend && key == lk;
        uint32_t v = same ? cnt : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane_id() == leader) flush_requests(c, lk, v);
        pend = pend && !same;
    }
}

__device__ inline void log_miss(ColdRef c, int32_t pix, int32_t k, const float p[3]) {
    const int32_t cap = c->misslog_cap;
    if (cap <= 0) return;
    const uint32_t i = atomicAdd(c->n_misslog, 1u);
    if ((int32_t)i < cap) {
        MissLogRec r;
        r.pix = pix;
        r.k = k;
        r.x = p[0];
        r.y = p[1];
        r.z = p[2];
        MissLogRec* log = c->misslog;
        log[i] = r;
    }
}

// Per-lane sample counters (32 bits per lane, summed per wave at the end);
// hits are the samples that are none of the other kinds.
struct Tally {
    uint32_t rays = 0, samples = 0, fallbacks = 0, misses = 0, skipped = 0;
    __device__ void add(int32_t st) {
        ++samples;
        if (st != S_HIT) {
            fallbacks += st == S_FALLBACK;
            misses += st == S_MISS;
            skipped += st == S_SKIP;
        }
    }
    // all 64 lanes of the wave must call this together; `lattice`: the
    // lattice mode's samples (gathered like misses) count as hits
    __device__ void commit(unsigned long long* stats, bool lattice = false) {
        const uint32_t m = lattice ? 0u : misses;
        wave_add_u64(&stats[ST_RAYS], rays);
        wave_add_u64(&stats[ST_SAMPLES], samples);
        wave_add_u64(&stats[ST_HITS], samples - fallbacks - m - skipped);
        wave_add_u64(&stats[ST_FALLBACKS], fallbacks);
        wave_add_u64(&stats[ST_MISSES], m);
        wave_add_u64(&stats[ST_SKIPPED], skipped);
    }
};

// Per-ray bookkeeping of one decided sample: request run-length aggregation
// (any sample not served at its own LoD requests its brick) and LRU stamps.
// The stochastic LoD makes a ray alternate between the bricks of two
// neighbouring LoDs, so runs are kept for the two keys requested last (one
// atomic per run when a third key comes, or at the end), and the two slots
// stamped last are remembered; a stamp is a plain store (every writer stores
// the same frame index).
struct RayBook {
    int32_t rk0 = -1, rk1 = -1;
    uint32_t rc0 = 0, rc1 = 0;
    int32_t ls0 = -1, ls1 = -1;
    __device__ void request(ColdRef c, int32_t key) {
        if (key == rk0) {
            ++rc0;
        } else if (key == rk1) {
            ++rc1;
        } else {
            flush_requests(c, rk1, rc1);
            rk1 = rk0;
            rc1 = rc0;
            rk0 = key;
            rc0 = 1;
        }
    }
    __device__ void note(const FrameDev& f, int32_t frame, ColdRef c, const SampleRes& s) {
        if (f.mode != CINR_CACHED || s.status == S_SKIP) return;
        if (s.status != S_HIT) request(c, s.req_key);
        if (s.slot >= 0 && s.slot != ls0 && s.slot != ls1) {
            f.last_used[s.slot] = frame;
            ls1 = ls0;
            ls0 = s.slot;
        }
    }
    // at the end of a ray, all 64 lanes together (see wave_flush_requests)
    __device__ void wave_flush(ColdRef c) {
        wave_flush_requests(c, rk0, rc0);
        wave_flush_requests(c, rk1, rc1);
        rk0 = rk1 = -1;
        rc0 = rc1 = 0;
    }
    // The same for scattered lookups (the path tracer): a stamp is stored
    // only when the slot does not hold it yet, so that lookups spread over
    // many slots do not dirty a cache line each.
    __device__ void note_scattered(const FrameDev& f, int32_t frame, ColdRef c, const SampleRes& s) {
        if (f.mode != CINR_CACHED || s.status == S_SKIP) return;
        if (s.status != S_HIT) request(c, s.req_key);
        if (s.slot >= 0 && s.slot != ls0 && s.slot != ls1) {
            if (f.last_used[s.slot] != frame) f.last_used[s.slot] = frame;
            ls1 = ls0;
            ls0 = s.slot;
        }
    }
};

__global__ __launch_bounds__(kBlock) void k_frame_begin(FrameDev f, int32_t n_ctr, const float* minmax,
                                                        int64_t n_cells, CacheCtr* cctr) {
    // bit r of nz: TF row r has a non-zero opacity (4 waves x 64 rows)
    __shared__ uint64_t nz[4];
    const uint64_t m = __ballot(f.tf[4 * threadIdx.x + 3] > 0.0f);
    if (lane_id() == 0) nz[threadIdx.x >> 6] = m;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    // the frame's camera, index and LoD seed: host block -> device (without a
    // host block, k_store_var stored them before this launch)
    if (f.var_src && t < 32) reinterpret_cast<uint32_t*>(f.var)[t] = reinterpret_cast<const uint32_t*>(f.var_src)[t];
    if (t == 0 && cctr) {
        cctr->frame = f.var_src ? f.var_src->frame : f.var->frame;
        cctr->n_views = (uint32_t)f.n_views;
    }
    if (t == 0 && f.view_table) f.view_table[f.view_index] = ViewEnd{f.stats, f.ctr, f.max_iters, 0};
    if (t == 0 && f.exit_ticket) *f.exit_ticket = 0u;
    if (t < n_ctr) f.ctr[t] = IterCtr{0u, 0u, 0u, 0u};
    if (t < 16) f.claim[t * kClaimStride] = 0u;
    if (t < ST_COUNT) f.stats[t] = 0ull;
    if (t == 0 && cctr) cctr->n_misslog = 0u;
    // macro-cell flags (Section 5.2): maximum opacity over the TF rows a
    // cell's value range can reach; zero means the cell is skipped.  That
    // maximum is positive exactly when one of the rows lo..hi has a positive
    // opacity, which the row bits answer a word at a time.  One bit per cell,
    // 64 cells (one wave) per word.
    if (f.flags && (t >> 6) < f.flag_words) {
        bool vis = false;
        if (t < n_cells) {
            const float a = minmax[2 * t] * 255.0f;
            const float b = minmax[2 * t + 1] * 255.0f;
            int32_t lo = (int32_t)__builtin_floorf(a), hi = (int32_t)__builtin_ceilf(b);
            lo = lo < 0 ? 0 : lo;
            hi = hi > 255 ? 255 : hi;
            for (int32_t w = lo >> 6; w <= (hi >> 6) && lo <= hi; ++w) {
                const int32_t a0 = lo > 64 * w ? lo - 64 * w : 0;
                const int32_t a1 = hi < 64 * w + 63 ? hi - 64 * w : 63;
                const uint64_t range = (~0ull << a0) & (~0ull >> (63 - a1));
                vis = vis || (nz[w] & range) != 0ull;
            }
        }
        const uint64_t word = __ballot(vis);
        if (lane_id() == 0) f.flags[t >> 6] = word;
    }
    // adaptive sampling rate: each cell's code from the exact maximum opacity
    // over its rows, through a sparse table (st[l][r]: rows r .. r + 2^l - 1)
    if (f.adapt > 0) {
        __shared__ float st[9][256];
        st[0][threadIdx.x] = f.tf[4 * threadIdx.x + 3];
        __syncthreads();
        for (int l = 1; l < 9; ++l) {
            const int r2 = (int)threadIdx.x + (1 << (l - 1));
            st[l][threadIdx.x] = fmaxf(st[l - 1][threadIdx.x], st[l - 1][r2 < 256 ? r2 : 255]);
            __syncthreads();
        }
        if (t < n_cells) {
            const float a = minmax[2 * t] * 255.0f;
            const float b = minmax[2 * t + 1] * 255.0f;
            int32_t lo = (int32_t)__builtin_floorf(a), hi = (int32_t)__builtin_ceilf(b);
            lo = lo < 0 ? 0 : lo;
            hi = hi > 255 ? 255 : hi;
            float mu = 0.0f;
            if (lo <= hi) {
                const int l = 31 - __builtin_clz((uint32_t)(hi - lo + 1));
                mu = fmaxf(st[l][lo], st[l][hi - (1 << l) + 1]);
            }
            f.cell_code[t] = mu > 0.0f ? (uint8_t)step_exp(mu, f.adapt) : (uint8_t)0xFFu;
        }
    }
}

// Work units of one march launch, claimed by waves.  Units are cut into
// 8*bands contiguous bands; XCD x (workgroups are dispatched round-robin over
// the 8 XCDs) claims bands x, x+8, ... in order through its own counter, so
// that each XCD's L2 sees compact image regions and every XCD gets bands from
// all over the image.  A wave whose XCD has no unit left claims from the
// others.  With `rev` the same sequence hands out unit n - 1 - u instead of u:
// a lockstep wave takes as long as its longest ray, and the tuner picks the
// direction that starts a view's tiles of long rays early rather than last.

struct UnitQueue {
    uint32_t* ctr;  // 8 counters, kClaimStride words apart
    uint32_t n_units, bsz, per_x, home;
    bool rev;           // units handed out from the last one down
    uint32_t dead = 0;  // counters known to be exhausted (wave-uniform)
    __device__ UnitQueue(uint32_t* c, uint32_t n, uint32_t bands, bool reverse) : ctr(c), n_units(n), rev(reverse) {
        const uint32_t nb = 8u * bands;
        bsz = (n + nb - 1u) / nb;
        per_x = bands * bsz;
        home = blockIdx.x & 7u;
    }
    // Next unit for the whole wave, or -1 when every counter is exhausted.
    // Each trip either returns, or advances a counter that is bounded by
    // per_x, or marks one of the 8 counters dead.
    __device__ int64_t claim() {
        while (dead != 0xFFu) {
            uint32_t xo = 0;
            while ((dead >> xo) & 1u) ++xo;
            const uint32_t x = (home + xo) & 7u;
            uint32_t j = 0;
            if (lane_id() == 0) j = atomicAdd(&ctr[x * kClaimStride], 1u);
            j = __builtin_amdgcn_readfirstlane(j);
            if (j >= per_x) {
                dead |= 1u << xo;
                continue;
            }
            const uint32_t band = x + 8u * (j / bsz);
            const uint32_t u = band * bsz + j % bsz;
            if (u < n_units) return (int64_t)(rev ? n_units - 1u - u : u);
        }
        return -1;
    }
};

// Persistent march: each wave claims work units of 64 rays (one per lane) and
// marches them in lockstep, so that neighbouring rays read neighbouring brick
// samples together.  Every lane of a wave runs the same trips of the unit loop
// so that list reservations can be made per wave.
// kWaves: waves per SIMD the register budget allows (3: up to 168 VGPRs, no
// spills; 4: 128 VGPRs with some spills but more latency hiding).  Neither
// wins everywhere (short rays favour 3, long ones 4), so the online tuner
// tries both.
// kAdapt: adaptive sampling rate (macro-cell codes instead of visibility
// bits); a sample of step exponent e is followed by sample k + 2^e.  kPool:
// the pool's storage (binary32, binary16, or mixed per LoD).
template <int kPipe, bool kLdsFlags, int kFast, bool kAdapt, int kPool, int kWaves>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWaves, 8))) void k_march(FrameDev f, int32_t it, uint32_t n0) {
    static_assert(!kAdapt || kPipe == 1, "the adaptive sampler decides one sample ahead at most");
    const FrameHot hot = load_hot(f.var);  // before any store of this kernel
    // a later iteration without rays (one queued before the count was known)
    // leaves at once; workgroup 0 still clears the next iteration's counters
    if (it > 0 && f.ctr[it].live == 0u) {
        if (blockIdx.x == 0 && threadIdx.x < 8) f.claim[(((it + 1) & 1) * 8 + threadIdx.x) * kClaimStride] = 0u;
        return;
    }
    // the pre-load frames march every ray to the end of the box (Sec. 4.3.4)
    const bool ert_on = f.ert_on && hot.preload == 0;
    __shared__ float4 tfs[256];
    __shared__ LodGeom lgs[kMaxLods];
    __shared__ uint64_t sflags[kLdsFlags ? (kAdapt ? kMaxLdsCells / 8 : kMaxLdsFlagWords) : 1];
    __shared__ int2 slotc[kSlotWays * kBlock];
    tfs[threadIdx.x] = reinterpret_cast<const float4*>(f.tf)[threadIdx.x];
    if (threadIdx.x < kMaxLods) lgs[threadIdx.x] = f.geo.lod[threadIdx.x];
#pragma unroll
    for (int w = 0; w < kSlotWays; ++w) slotc[w * kBlock + threadIdx.x] = make_int2(-1, -1);
    if (kLdsFlags) {
        if (kAdapt) {
            const uint64_t* src = reinterpret_cast<const uint64_t*>(f.cell_code);
            for (int32_t w = threadIdx.x; w < (f.n_cells + 7) / 8; w += kBlock) sflags[w] = src[w];
        } else {
            for (int32_t w = threadIdx.x; w < f.flag_words; w += kBlock) sflags[w] = f.flags[w];
        }
    }
    // the counters of the next iteration were last used two launches ago
    if (blockIdx.x == 0 && threadIdx.x < 8) f.claim[(((it + 1) & 1) * 8 + threadIdx.x) * kClaimStride] = 0u;
    __syncthreads();
    using Flags = typename std::conditional<
        kAdapt, typename std::conditional<kLdsFlags, LdsCodes, GlobalCodes>::type,
        typename std::conditional<kLdsFlags, LdsFlags, GlobalFlags>::type>::type;
    Flags fl;
    if constexpr (kAdapt)
        fl.c = kLdsFlags ? reinterpret_cast<const uint8_t*>(sflags) : f.cell_code;
    else
        fl.w = kLdsFlags ? (const uint64_t*)sflags : (const uint64_t*)f.flags;

    // iteration 0: all pixels in 8x8 tiles (unit = tile); later: the rays
    // re-queued by k_shade, 64 per unit
    __shared__ MarchCold cold_s;
    if (threadIdx.x == 0) {
        MarchCold& c = cold_s;
        c.cam = f.var->cam;
        c.rgba = f.rgba;
        c.k_next = f.k_next;
        c.cur = (it & 1) ? f.live1 : f.live0;
        c.pend_pix = f.pend_pix;
        c.pend_n = f.pend_n;
        c.vals = f.vals;
        c.miss_rec = f.miss_rec;
        c.pending = &f.ctr[it].pending;
        c.misses = &f.ctr[it].misses;
        c.misslog = f.misslog;
        c.n_misslog = f.n_misslog;
        c.misslog_cap = f.misslog_cap;
        c.req = f.req ? f.req + f.key_base : nullptr;
        c.touched = f.touched;
        c.n_touched = f.n_touched;
        c.key_base = f.key_base;
        c.ert_rec = f.ert_rec;
    }
    __syncthreads();
    const ColdRef cold = &cold_s;
    const uint32_t n = it == 0 ? n0 : f.ctr[it].live;
    UnitQueue q(f.claim + (it & 1) * 8 * kClaimStride, (n + 63u) / 64u, (uint32_t)f.xcd_bands, f.claim_rev != 0);
    const int32_t S = f.S;
    const bool lat = f.mode == CINR_UNCACHED_LATTICE;
    const int32_t Sg = lat ? S / 8 : S;  // samples gathered per pending step
    Tally tally;
    SlotCache sc{&slotc[threadIdx.x]};  // residency is constant within a frame: valid across rays
    for (;;) {
        const int64_t unit = q.claim();
        if (unit < 0) break;
        const uint32_t r = (uint32_t)unit * 64u + (uint32_t)lane_id();
        bool has = r < n;
        int32_t pix = 0;
        float o[3], d[3], ts = 0.0f, te = -1.0f;
        if (has) {
            const CamDev cam = load_cam(cold->cam);
            int32_t i, j;
            if (it == 0) {
                const uint32_t tiles_x = (uint32_t)(cam.W + 7) / 8u;
                const uint32_t tile = r >> 6, w = r & 63u;
                i = (int32_t)(tile % tiles_x) * 8 + (int32_t)(w & 7u);
                j = (int32_t)(tile / tiles_x) * 8 + (int32_t)(w >> 3);
                has = i < cam.W && j < cam.H;
            } else {
                const int32_t* cur = cold->cur;
                pix = cur[r];
                i = pix % cam.W;
                j = pix / cam.W;
            }
            if (has) {
                if (it == 0) pix = j * cam.W + i;
                const bool hit = ray_setup(cam, f.vm1, i, j, o, d, ts, te);
                if (it == 0) {
                    float4* rgba = cold->rgba;
                    if (!hit) rgba[pix] = make_float4(0.f, 0.f, 0.f, 0.f);
                    int32_t* rec = cold->ert_rec;
                    if (rec) rec[pix] = -1;
                    tally.rays += hit;
                }
                has = hit;
            }
        }
        if (__ballot(has) == 0ull) continue;
        int32_t k = 0;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        if (has && it > 0) {
            const int32_t* kn = cold->k_next;
            const float4* rgba = cold->rgba;
            k = kn[pix];
            acc = rgba[pix];
        }
        RayBook book;
        bool pend = false;
        int32_t e_miss = 0;  // step exponent of the sample that missed
        if (has) {
            // Fast phase, software-pipelined: decide and fetch a group of
            // kPipe samples, then commit them in order (bookkeeping,
            // compositing, early termination).  Samples fetched past an early
            // termination or a true miss are discarded without side effects.
            float p[3];
            bool run = true;
            while (run) {
                SampleRes grp[kPipe];
                int32_t cnt = 0;
#pragma unroll
                for (int u = 0; u < kPipe; ++u) {
                    if (cnt == u && sample_pos(o, d, ts, te, f.step, k + u, f.vm1, p)) {
                        grp[u] = sample_cache<kFast, kAdapt, kPool>(f, hot, lgs, fl, p, sc);
                        ++cnt;
                    }
                }
                if (cnt < kPipe) run = false;
#pragma unroll
                for (int u = 0; u < kPipe; ++u) {
                    if (u >= cnt) break;
                    const SampleRes& sr = grp[u];
                    tally.add(sr.status);
                    book.note(f, hot.frame, cold, sr);
                    if (sr.status == S_MISS) {
                        pend = true;
                        run = false;
                        e_miss = sr.e;
                        break;
                    }
                    if (sr.status != S_SKIP)
                        composite(acc, sr.value, tfs, kAdapt ? __builtin_ldexpf(f.step, sr.e) : f.step);
                    k += kAdapt ? (1 << sr.e) : 1;
                    if (ert_on && acc.w >= f.ert) {
                        int32_t* rec = cold->ert_rec;
                        if (rec) rec[pix] = k;
                        run = false;
                        break;
                    }
                }
            }
        }
        // a wavefront step of S samples starting at the miss (the lattice
        // mode: S / 8 samples, whose 8 lattice corners each take a value slot)
        if (__ballot(pend) != 0ull) {
            const uint32_t pi = wave_reserve(pend ? 1u : 0u, cold->pending);
            uint64_t mask = 0;
            int32_t nc = 0;
            if (pend) {
                int32_t* pp = cold->pend_pix;
                pp[pi] = pix;
                float* vb = cold->vals + (int64_t)pi * S;
                uint8_t* ve = f.vexp + (int64_t)pi * S;  // adaptive: each sample's step exponent
                if (kAdapt) ve[0] = (uint8_t)e_miss;
                mask = 1;
                nc = 1;
                int32_t kg = k + (kAdapt ? (1 << e_miss) : 1);  // grid index of the next sample
                while (nc < Sg) {
                    float qp[3];
                    if (!sample_pos(o, d, ts, te, f.step, kg, f.vm1, qp)) break;
                    const SampleRes sr = sample_cache<kFast, kAdapt, kPool>(f, hot, lgs, fl, qp, sc);
                    tally.add(sr.status);
                    book.note(f, hot.frame, cold, sr);
                    if (sr.status == S_MISS)
                        mask |= 1ull << nc;
                    else
                        vb[lat ? 8 * nc : nc] = sr.status == S_SKIP ? -1.0f : sr.value;
                    if (kAdapt) ve[nc] = (uint8_t)sr.e;
                    kg += kAdapt ? (1 << sr.e) : 1;
                    ++nc;
                }
                int32_t* pn = cold->pend_n;
                int32_t* kn = cold->k_next;
                pn[pi] = nc;
                kn[pix] = k;
            }
            // true-miss records (position, destination slot), reserved per wave
            uint32_t mb = wave_reserve((uint32_t)__popcll(mask) * (lat ? 8u : 1u), cold->misses);
            if (pend) {
                float4* mr = cold->miss_rec;
                const uint8_t* ve = f.vexp + (int64_t)pi * S;
                int32_t kg = k;  // grid index of gathered sample sidx
                for (int32_t sidx = 0; sidx < nc; ++sidx) {
                    if ((mask >> sidx) & 1ull) {
                        float qp[3];
                        sample_pos(o, d, ts, te, f.step, kg, f.vm1, qp);
                        if (lat) {
                            // the 8 LoD-0 lattice points around the sample (cell
                            // clamped so that its upper corner exists)
                            int32_t j[3];
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                j[a] = (int32_t)qp[a];
                                if (j[a] > f.dims[a] - 2) j[a] = f.dims[a] - 2;
                            }
                            for (int32_t n = 0; n < 8; ++n)
                                mr[mb++] = make_float4((float)(j[0] + (n & 1)), (float)(j[1] + ((n >> 1) & 1)),
                                                       (float)(j[2] + (n >> 2)),
                                                       __uint_as_float(pi * (uint32_t)S + (uint32_t)(8 * sidx + n)));
                        } else {
                            mr[mb++] = make_float4(qp[0], qp[1], qp[2], __uint_as_float(pi * (uint32_t)S + (uint32_t)sidx));
                        }
                        log_miss(cold, pix, kg, qp);
                    }
                    kg += kAdapt ? (1 << ve[sidx]) : 1;
                }
            }
        }
        book.wave_flush(cold);
        if (has) {
            float4* rgba = cold->rgba;
            rgba[pix] = acc;
        }
    }
    tally.commit(f.stats, lat);
    if (it == 0 && f.gather_host) {
        // the frame's pending count once every workgroup has finished: the
        // last one to take a ticket reads it (all reservations precede the
        // fences) and hands it to the host and to the frame-end gate
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            const uint32_t ticket = atomicAdd(f.exit_ticket, 1u);
            if (ticket == gridDim.x - 1u) {
                __threadfence();
                const uint32_t pending = atomicAdd(&f.ctr[0].pending, 0u);
                f.gather_host[f.view_index] = pending;
                *f.gather_gate = pending == 0u ? 1u : 0u;
                __threadfence_system();
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_shade(FrameDev f, int32_t it) {
    if (f.ctr[it].pending == 0u) return;  // nothing to shade (the same for every workgroup)
    const CamDev cam = f.var->cam;
    __shared__ float4 tfs[256];
    tfs[threadIdx.x] = reinterpret_cast<const float4*>(f.tf)[threadIdx.x];
    __syncthreads();
    const uint32_t n = f.ctr[it].pending;
    int32_t* next = (it & 1) ? f.live0 : f.live1;
    const int32_t S = f.S;
    const bool ert_on = f.ert_on && f.var->preload == 0;  // suspended in the pre-load frames
    const bool lat = f.mode == CINR_UNCACHED_LATTICE;
    for (uint32_t pi = blockIdx.x * kBlock + threadIdx.x; pi < n; pi += gridDim.x * kBlock) {
        const int32_t pix = f.pend_pix[pi];
        const int32_t nc = f.pend_n[pi];
        int32_t k = f.k_next[pix];
        float4 acc = f.rgba[pix];
        const float* vb = f.vals + (int64_t)pi * S;
        const uint8_t* ve = f.vexp + (int64_t)pi * S;
        bool done = false;
        int32_t kg = k;  // grid index after the composited samples
        float lo[3] = {0.f, 0.f, 0.f}, ld[3] = {0.f, 0.f, 0.f}, lts = 0.0f, lte = -1.0f;
        if (lat) ray_setup(cam, f.vm1, pix % f.W, pix / f.W, lo, ld, lts, lte);
        for (int32_t s = 0; s < nc; ++s) {
            float v;
            if (lat) {
                // trilinear of the sample's 8 lattice values (a skipped sample
                // holds -1 in its first slot)
                const float* c = vb + 8 * s;
                v = c[0];
                if (v >= 0.0f) {
                    float q[3];
                    sample_pos(lo, ld, lts, lte, f.step, kg, f.vm1, q);
                    float fr[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        int32_t j = (int32_t)q[a];
                        if (j > f.dims[a] - 2) j = f.dims[a] - 2;
                        fr[a] = q[a] - (float)j;
                    }
                    const float x00 = __builtin_fmaf(fr[0], c[1] - c[0], c[0]);
                    const float x10 = __builtin_fmaf(fr[0], c[3] - c[2], c[2]);
                    const float x01 = __builtin_fmaf(fr[0], c[5] - c[4], c[4]);
                    const float x11 = __builtin_fmaf(fr[0], c[7] - c[6], c[6]);
                    const float y0 = __builtin_fmaf(fr[1], x10 - x00, x00);
                    const float y1 = __builtin_fmaf(fr[1], x11 - x01, x01);
                    v = __builtin_fmaf(fr[2], y1 - y0, y0);
                }
            } else {
                v = vb[s];
            }
            const int32_t e = f.adapt > 0 ? (int32_t)ve[s] : 0;
            if (v >= 0.0f) composite(acc, v, tfs, e ? __builtin_ldexpf(f.step, e) : f.step);
            kg += 1 << e;
            if (ert_on && acc.w >= f.ert) {
                if (f.ert_rec) f.ert_rec[pix] = kg;
                done = true;
                break;
            }
        }
        if (!done) {
            k = kg;
            const int32_t i = pix % f.W, j = pix / f.W;
            float o[3], d[3], ts, te;
            ray_setup(cam, f.vm1, i, j, o, d, ts, te);
            float q[3];
            if (sample_pos(o, d, ts, te, f.step, k, f.vm1, q)) {
                const int64_t li = wave_append(true, &f.ctr[it + 1].live);
                next[li] = pix;
                f.k_next[pix] = k;
            }
        }
        f.rgba[pix] = acc;
    }
}

// ---------------------------------------------------------------------------
// Path tracing (Section 5.1): the second wavefront pipeline, Woodcock delta
// tracking through the same sampler.  One lane per pixel runs the pixel's
// paths one after the other until they are done or a tentative collision is a
// true miss; then the next tentative collisions of the segment (up to
// `gather`, those before its end) are looked up too, their misses queued for
// inference straight into the pixel's state, and the pixel resumes in the
// next iteration.  Lookups count, request and stamp exactly as the ray
// marcher's samples.
// ---------------------------------------------------------------------------

// TF at v (rows floor(255 v) and the next, each interpolation rounded once),
// opacity clamped to [0, 1]: the lookup of the compositing step.
__device__ inline float4 tf_at(const float4* tfs, float v) {
    const float x = v * 255.0f;
    int32_t i0 = (int32_t)x;
    i0 = i0 > 254 ? 254 : (i0 < 0 ? 0 : i0);
    const float t = x - (float)i0;
    const float4 a = tfs[i0], b = tfs[i0 + 1];
    float4 r;
    r.x = __builtin_fmaf(t, b.x - a.x, a.x);
    r.y = __builtin_fmaf(t, b.y - a.y, a.y);
    r.z = __builtin_fmaf(t, b.z - a.z, a.z);
    r.w = __builtin_fmaf(t, b.w - a.w, a.w);
    r.w = r.w < 0.0f ? 0.0f : (r.w > 1.0f ? 1.0f : r.w);
    return r;
}

// A pixel's paths in registers (PtState without the gathered values, which
// are read from memory as they are consumed).
struct PtLane {
    float o[3], d[3], t, te, beta[3], lp[3], sum[3];
    uint32_t n, path, done, hits, kind, nc, gi;

    __device__ void load(const PtState& g) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = g.o[a];
            d[a] = g.d[a];
            beta[a] = g.beta[a];
            lp[a] = g.lp[a];
            sum[a] = g.sum[a];
        }
        t = g.t;
        te = g.te;
        n = g.n;
        path = g.path;
        done = g.done;
        hits = g.hits;
        kind = g.kind;
        nc = g.nc;
        gi = 0;
    }
    __device__ void store(PtState& g) const {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            g.o[a] = o[a];
            g.d[a] = d[a];
            g.beta[a] = beta[a];
            g.lp[a] = lp[a];
            g.sum[a] = sum[a];
        }
        g.t = t;
        g.te = te;
        g.n = n;
        g.path = path;
        g.done = done;
        g.hits = hits;
        g.kind = kind;
        g.nc = nc;
    }
    // a new path: the primary ray's segment (false when it misses the box)
    __device__ bool begin(const CamDev& cam, const float vm1[3], int32_t i, int32_t j) {
        float ts, te_;
        const bool hit = ray_setup<true>(cam, vm1, i, j, o, d, ts, te_);
        t = ts;
        te = te_;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            beta[a] = 1.0f;
            lp[a] = 0.0f;
        }
        kind = PT_PRIMARY;
        nc = gi = 0;
        return hit;
    }
    // a new segment from o along dir
    __device__ void segment(const float dir[3], uint32_t k, const float vm1[3]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] = dir[a];
        t = 0.0f;
        te = pt_segment_exit(o, d, vm1);
        kind = (kind & ~3u) | k;
        nc = gi = 0;
    }
};

// The lane's pixel after its last path (or the event budget): the mean over
// the completed paths.
__device__ inline float4 pt_pixel_value(const PtLane& s) {
    if (s.done == 0) return make_float4(0.f, 0.f, 0.f, 0.f);
    const float J = (float)s.done;
    return make_float4(s.sum[0] / J, s.sum[1] / J, s.sum[2] / J, (float)s.hits / J);
}

// (3 waves per SIMD: 158 VGPRs without spills; 4 would spill)
template <bool kLdsFlags, int kFast, int kPool>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_path(FrameDev f, int32_t it, uint32_t n0) {
    const FrameHot hot = load_hot(f.var);  // before any store of this kernel
    // as k_march: a later iteration without pixels leaves at once
    if (it > 0 && f.ctr[it - 1].pending == 0u) {
        if (blockIdx.x == 0 && threadIdx.x < 8) f.claim[(((it + 1) & 1) * 8 + threadIdx.x) * kClaimStride] = 0u;
        return;
    }
    __shared__ float4 tfs[256];
    __shared__ LodGeom lgs[kMaxLods];
    __shared__ uint64_t sflags[kLdsFlags ? kMaxLdsFlagWords : 1];
    __shared__ int2 slotc[kSlotWays * kBlock];
    tfs[threadIdx.x] = reinterpret_cast<const float4*>(f.tf)[threadIdx.x];
    if (threadIdx.x < kMaxLods) lgs[threadIdx.x] = f.geo.lod[threadIdx.x];
#pragma unroll
    for (int w = 0; w < kSlotWays; ++w) slotc[w * kBlock + threadIdx.x] = make_int2(-1, -1);
    if (kLdsFlags)
        for (int32_t w = threadIdx.x; w < f.flag_words; w += kBlock) sflags[w] = f.flags[w];
    // the counters of the next iteration were last used two launches ago
    if (blockIdx.x == 0 && threadIdx.x < 8) f.claim[(((it + 1) & 1) * 8 + threadIdx.x) * kClaimStride] = 0u;
    __shared__ MarchCold cold_s;
    if (threadIdx.x == 0) {
        MarchCold& c = cold_s;
        c.cam = f.var->cam;
        c.rgba = f.rgba;
        c.pending = &f.ctr[it].pending;
        c.misses = &f.ctr[it].misses;
        c.miss_rec = f.miss_rec;
        c.misslog = f.misslog;
        c.n_misslog = f.n_misslog;
        c.misslog_cap = f.misslog_cap;
        c.req = f.req ? f.req + f.key_base : nullptr;
        c.touched = f.touched;
        c.n_touched = f.n_touched;
        c.key_base = f.key_base;
    }
    __syncthreads();
    using Flags = typename std::conditional<kLdsFlags, LdsFlags, GlobalFlags>::type;
    Flags fl;
    fl.w = kLdsFlags ? (const uint64_t*)sflags : (const uint64_t*)f.flags;
    const ColdRef cold = &cold_s;
    // iteration 0: all pixels in 8x8 tiles; later: the pixels left waiting
    // by the previous iteration
    const uint32_t n = it == 0 ? n0 : f.ctr[it - 1].pending;
    const int32_t* cur = (it & 1) ? f.live1 : f.live0;
    int32_t* next = (it & 1) ? f.live0 : f.live1;
    UnitQueue q(f.claim + (it & 1) * 8 * kClaimStride, (n + 63u) / 64u, (uint32_t)f.xcd_bands, f.claim_rev != 0);
    const PtDev P = f.path;
    const uint32_t key1 = (uint32_t)hot.frame;
    Tally tally;
    SlotCache sc{&slotc[threadIdx.x]};  // residency is constant within a frame
    for (;;) {
        const int64_t unit = q.claim();
        if (unit < 0) break;
        const uint32_t r = (uint32_t)unit * 64u + (uint32_t)lane_id();
        bool has = r < n;
        int32_t pix = 0, pi_ = 0, pj = 0;
        PtLane s;
        bool begin_path = false;  // the pixel's next path starts at the top of the event loop
        if (has) {
            const CamDev cam = load_cam(cold->cam);
            if (it == 0) {
                const uint32_t tiles_x = (uint32_t)(cam.W + 7) / 8u;
                const uint32_t tile = r >> 6, w = r & 63u;
                pi_ = (int32_t)(tile % tiles_x) * 8 + (int32_t)(w & 7u);
                pj = (int32_t)(tile / tiles_x) * 8 + (int32_t)(w >> 3);
                has = pi_ < cam.W && pj < cam.H;
                if (has) {
                    pix = pj * cam.W + pi_;
                    s.n = s.path = s.done = s.hits = 0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) s.sum[a] = 0.0f;
                    begin_path = true;
                }
            } else {
                pix = cur[r];
                pi_ = pix % cam.W;
                pj = pix / cam.W;
                s.load(P.st[pix]);
            }
        }
        if (__ballot(has) == 0ull) continue;
        RayBook book;
        bool pend = false, fin = false;
        float t_miss = 0.0f;  // t of the tentative collision that missed
        if (has) {
            const float* gvals = P.st[pix].vals;
            while (!fin && !pend) {
                if (begin_path) {
                    // the one place where a pixel's primary ray is set up
                    begin_path = false;
                    const CamDev cam = load_cam(cold->cam);
                    const bool hit = s.begin(cam, f.vm1, pi_, pj);
                    if (s.path == 0) {
                        tally.rays += hit;
                        if (!hit) {  // a ray that misses the box: no paths
                            fin = true;
                            break;
                        }
                    }
                }
                if (s.n >= kPtMaxEvents) {  // budget spent: the path in progress is dropped
                    fin = true;
                    break;
                }
                const uint32_t e = s.n;
                uint32_t w[4] = {(uint32_t)pix, e, 0u, 0u};
                philox4x32_10(w, P.seed, key1);
                const float step = pt_free_flight(w[0]) * P.inv_sigma;
                const float t = s.t + step;
                const uint32_t kind = s.kind & 3u;
                bool collided = false;
                float v = 0.0f;
                float p[3];
                if (t > s.te) {
                    s.n = e + 1;
                    s.t = t;
                } else {
                    pt_pos(s.o, s.d, t, f.vm1, p);
                    bool skip;
                    if (s.gi < s.nc) {
                        v = gvals[s.gi];
                        ++s.gi;
                        skip = v < 0.0f;
                    } else {
                        const SampleRes sr = sample_cache<kFast, false, kPool>(f, hot, lgs, fl, p, sc);
                        tally.add(sr.status);
                        book.note_scattered(f, hot.frame, cold, sr);
                        if (sr.status == S_MISS) {
                            pend = true;  // s.n and s.t stay before event e
                            t_miss = t;
                            break;
                        }
                        skip = sr.status == S_SKIP;
                        v = sr.value;
                    }
                    s.n = e + 1;
                    s.t = t;
                    const float alpha = skip ? 0.0f : tf_at(tfs, v).w;
                    if (pt_uniform(w[1]) >= alpha) continue;  // null collision
                    collided = true;
                }
                // the segment ends: a real collision at p, or the segment is left
                bool after_shadow = false;
                if (collided && kind != PT_SHADOW) {
                    if (kind == PT_PRIMARY) s.kind |= 1u << 31;
                    const float4 c = tf_at(tfs, v);
                    s.beta[0] *= c.x;
                    s.beta[1] *= c.y;
                    s.beta[2] *= c.z;
#pragma unroll
                    for (int a = 0; a < 3; ++a) s.o[a] = p[a];
                    s.segment(P.ldir, PT_SHADOW, f.vm1);
                    continue;
                }
                bool path_end = false;
                if (collided) {  // the shadow ray is blocked
                    after_shadow = true;
                } else if (kind == PT_SHADOW) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) s.lp[a] = __builtin_fmaf(s.beta[a], P.light[a], s.lp[a]);
                    after_shadow = true;
                } else {
                    if (kind == PT_SCATTER)
#pragma unroll
                        for (int a = 0; a < 3; ++a) s.lp[a] = __builtin_fmaf(s.beta[a], P.ambient[a], s.lp[a]);
                    path_end = true;
                }
                if (after_shadow) {
                    const uint32_t bounce = ((s.kind >> 2) & 0xFFFFu) + 1u;
                    s.kind = (s.kind & ~(0xFFFFu << 2)) | (bounce << 2);
                    if ((int32_t)bounce == P.bounces) {
                        path_end = true;
                    } else {
                        // isotropic scattering from the collision (the shadow ray's origin)
                        float dir[3];
                        bool ok = false;
                        while (!ok) {
                            if (s.n >= kPtMaxEvents) break;
                            uint32_t wd[4] = {(uint32_t)pix, s.n, 0u, 0u};
                            philox4x32_10(wd, P.seed, key1);
                            ++s.n;
                            ok = pt_marsaglia(wd, dir);
                        }
                        if (!ok) {
                            fin = true;
                            break;
                        }
                        s.segment(dir, PT_SCATTER, f.vm1);
                    }
                }
                if (path_end) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) s.sum[a] += s.lp[a];
                    s.hits += s.kind >> 31;
                    s.done += 1;
                    s.path += 1;
                    if ((int32_t)s.path == P.spp)
                        fin = true;
                    else
                        begin_path = true;
                }
            }
        }
        // a true miss: look up the next tentative collisions of the segment
        // as well, then queue the pixel and its misses
        uint64_t mask = 0;
        uint32_t nc = 0;
        if (pend) {
            float* sv = P.st[pix].vals;
            mask = 1;
            nc = 1;
            float tg = t_miss;
            while ((int32_t)nc < P.gather) {
                uint32_t w[4] = {(uint32_t)pix, s.n + nc, 0u, 0u};
                philox4x32_10(w, P.seed, key1);
                const float t2 = tg + pt_free_flight(w[0]) * P.inv_sigma;
                if (t2 > s.te) break;
                tg = t2;
                float p[3];
                pt_pos(s.o, s.d, tg, f.vm1, p);
                const SampleRes sr = sample_cache<kFast, false, kPool>(f, hot, lgs, fl, p, sc);
                tally.add(sr.status);
                book.note_scattered(f, hot.frame, cold, sr);
                if (sr.status == S_MISS)
                    mask |= 1ull << nc;
                else
                    sv[nc] = sr.status == S_SKIP ? -1.0f : sr.value;
                ++nc;
            }
            s.nc = nc;
        }
        const uint32_t qi = wave_reserve(pend ? 1u : 0u, cold->pending);
        uint32_t mb = wave_reserve(pend ? (uint32_t)__popcll(mask) : 0u, cold->misses);
        if (pend) {
            next[qi] = pix;
            float4* mr = cold->miss_rec;
            float tg = s.t;
            for (uint32_t k = 0; k < nc; ++k) {
                uint32_t w[4] = {(uint32_t)pix, s.n + k, 0u, 0u};
                philox4x32_10(w, P.seed, key1);
                tg = tg + pt_free_flight(w[0]) * P.inv_sigma;
                if ((mask >> k) & 1ull) {
                    float p[3];
                    pt_pos(s.o, s.d, tg, f.vm1, p);
                    const uint32_t dst = (uint32_t)pix * 32u + (uint32_t)kPtValsWord + k;
                    mr[mb++] = make_float4(p[0], p[1], p[2], __uint_as_float(dst));
                    log_miss(cold, pix, (int32_t)(s.n + k), p);
                }
            }
            s.store(P.st[pix]);
        }
        book.wave_flush(cold);
        if (has) {
            if (fin) {
                float4* rgba = cold->rgba;
                rgba[pix] = pt_pixel_value(s);
            }
        }
    }
    tally.commit(f.stats);
}

// Frame statistics of one view; the cache manager's counters are those of the
// whole frame (all views).  `reset` (the last view) clears the request list.
// The view ran march launches 0 .. n-1, where n - 1 is the first iteration
// that left no ray pending, or max_iters - 1.
__global__ void k_frame_end(FrameDev f, int32_t max_iters, CacheCtr* cctr, int32_t reset, const uint32_t* gate) {
    if (gate && *gate == 0u) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int32_t n = 1;
        while (n < max_iters && f.ctr[n - 1].pending != 0u) ++n;
        f.stats[ST_ITERS] = (unsigned long long)n;
        if (cctr) {
            f.stats[ST_REQUESTED] = cctr->n_touched;
            f.stats[ST_SELECTED] = cctr->n_sel;
            f.stats[ST_EVICTED] = cctr->need_evict;
            if (reset) cctr->n_touched = 0u;  // the next frame's requests start empty
        }
    }
}

// ---------------------------------------------------------------------------

static int blocks_for(int64_t n, int64_t cap) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t launch_frame_begin(const FrameDev& f, int32_t n_iter_ctr, const float* minmax, int64_t n_cells,
                              CacheCtr* cctr, hipStream_t s) {
    int64_t n = n_iter_ctr;
    const bool cells = f.flags || f.adapt > 0;
    if (cells && n_cells > n) n = n_cells;
    if (n < ST_COUNT) n = ST_COUNT;
    hipLaunchKernelGGL(k_frame_begin, dim3(blocks_for(n, 1 << 20)), dim3(kBlock), 0, s, f, n_iter_ctr, minmax,
                       cells ? n_cells : 0, cctr);
    return hipGetLastError();
}

// Workgroups of one k_march instantiation that are resident at once on the
// current device (the grid of the persistent kernel), cached per device.
// Whether every byte offset into the pool fits in 32 bits (the uncached
// mode reads no pool).
static bool small_pool(const FrameDev& f, int pool_kind) {
    const uint64_t brick_bytes = (uint64_t)f.geo.brick * f.geo.brick * f.geo.brick * (pool_kind == POOL_F16 ? 2u : 4u);
    return f.mode != CINR_CACHED || (uint64_t)f.pool_bricks * brick_bytes < (1ull << 32);
}

template <int P, bool LDS, int FAST, bool A, int H, int W>
static hipError_t resident_blocks(int* out) {
    static int cache[64] = {0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (cache[dev] == 0) {
        int per_cu = 0, n_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_march<P, LDS, FAST, A, H, W>, kBlock, 0);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        cache[dev] = (per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1);
    }
    *out = cache[dev];
    return hipSuccess;
}

template <int P, bool LDS, int FAST, bool A, int H, int W>
static hipError_t launch_march_t(const FrameDev& f, int it, int64_t max_rays, uint32_t n0, hipStream_t s) {
    int cap = 0;
    hipError_t e = resident_blocks<P, LDS, FAST, A, H, W>(&cap);
    if (e != hipSuccess) return e;
    // one work unit (64 rays) per wave at least
    int64_t b = (max_rays + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    hipLaunchKernelGGL((k_march<P, LDS, FAST, A, H, W>), dim3((unsigned)b), dim3(kBlock), 0, s, f, it, n0);
    return hipGetLastError();
}

template <int P, bool LDS, bool A, int H, int W>
static hipError_t launch_march_l(const FrameDev& f, int it, int64_t max_rays, uint32_t n0, hipStream_t s) {
    // 16^3 bricks (or the uncached mode, which reads no pool) and 16^3
    // macro-cells (or none); 32-bit pool offsets below 4 GiB
    const bool cells = A || f.flags;
    const bool fast = (f.mode != CINR_CACHED || f.geo.brick == 16) && (!cells || f.mc_N == 16);
    if (fast && small_pool(f, H)) return launch_march_t<P, LDS, 1, A, H, W>(f, it, max_rays, n0, s);
    if (fast) return launch_march_t<P, LDS, 2, A, H, W>(f, it, max_rays, n0, s);
    return launch_march_t<P, LDS, 0, A, H, W>(f, it, max_rays, n0, s);
}

template <int P, bool A, int H, int W>
static hipError_t launch_march_p(const FrameDev& f, int it, int64_t max_rays, uint32_t n0, hipStream_t s) {
    const bool lds = A ? f.n_cells <= kMaxLdsCells : (f.flags && f.flag_words <= kMaxLdsFlagWords);
    if (lds) return launch_march_l<P, true, A, H, W>(f, it, max_rays, n0, s);
    return launch_march_l<P, false, A, H, W>(f, it, max_rays, n0, s);
}

template <int H, int W>
static hipError_t launch_march_w(const FrameDev& f, int it, int64_t n, uint32_t n0, hipStream_t s) {
    // the adaptive sampler decides its next sample after the current one
    if (f.adapt > 0) return launch_march_p<1, true, H, W>(f, it, n, n0, s);
    // kPipe: samples decided and fetched ahead per ray (8 runs as 4)
    switch (f.pipe) {
        case 1: return launch_march_p<1, false, H, W>(f, it, n, n0, s);
        case 2: return launch_march_p<2, false, H, W>(f, it, n, n0, s);
        default: return launch_march_p<4, false, H, W>(f, it, n, n0, s);
    }
}

template <int H>
static hipError_t launch_march_h(const FrameDev& f, int it, int64_t n, uint32_t n0, hipStream_t s) {
    if (f.waves == 4) return launch_march_w<H, 4>(f, it, n, n0, s);
    return launch_march_w<H, 3>(f, it, n, n0, s);
}

// The path tracer's persistent grid, as resident_blocks for k_march.
template <bool LDS, int FAST, int H>
static hipError_t launch_path_t(const FrameDev& f, int it, int64_t max_px, uint32_t n0, hipStream_t s) {
    static int cache[64] = {0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (cache[dev] == 0) {
        int per_cu = 0, n_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_path<LDS, FAST, H>, kBlock, 0);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        cache[dev] = (per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1);
    }
    int64_t b = (max_px + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cache[dev]) b = cache[dev];
    hipLaunchKernelGGL((k_path<LDS, FAST, H>), dim3((unsigned)b), dim3(kBlock), 0, s, f, it, n0);
    return hipGetLastError();
}

template <int H>
static hipError_t launch_path_h(const FrameDev& f, int it, int64_t n, uint32_t n0, hipStream_t s) {
    const bool fast = (f.mode != CINR_CACHED || f.geo.brick == 16) && (!f.flags || f.mc_N == 16);
    const int kind = fast ? (small_pool(f, H) ? 1 : 2) : 0;
    const bool lds = f.flags && f.flag_words <= kMaxLdsFlagWords;
    if (lds) {
        if (kind == 1) return launch_path_t<true, 1, H>(f, it, n, n0, s);
        if (kind == 2) return launch_path_t<true, 2, H>(f, it, n, n0, s);
        return launch_path_t<true, 0, H>(f, it, n, n0, s);
    }
    if (kind == 1) return launch_path_t<false, 1, H>(f, it, n, n0, s);
    if (kind == 2) return launch_path_t<false, 2, H>(f, it, n, n0, s);
    return launch_path_t<false, 0, H>(f, it, n, n0, s);
}

hipError_t launch_march(const FrameDev& f, int it, int64_t max_rays, hipStream_t s) {
    // iteration 0 walks all pixels in 8x8 tiles; later iterations at most
    // `max_rays` re-queued rays
    const uint32_t n0 = (uint32_t)(((f.W + 7) / 8) * ((f.H + 7) / 8)) * 64u;
    const int64_t n = it == 0 ? (int64_t)n0 : max_rays;
    if (f.path.on) {
        if (f.pool_kind == POOL_MIXED) return launch_path_h<POOL_MIXED>(f, it, n, n0, s);
        if (f.pool_kind == POOL_F16) return launch_path_h<POOL_F16>(f, it, n, n0, s);
        return launch_path_h<POOL_F32>(f, it, n, n0, s);
    }
    if (f.pool_kind == POOL_MIXED) return launch_march_h<POOL_MIXED>(f, it, n, n0, s);
    if (f.pool_kind == POOL_F16) return launch_march_h<POOL_F16>(f, it, n, n0, s);
    return launch_march_h<POOL_F32>(f, it, n, n0, s);
}

hipError_t launch_shade(const FrameDev& f, int it, int64_t cap_rays, hipStream_t s) {
    // the path tracer consumes its gathered values in its next march launch
    if (f.path.on) return hipSuccess;
    hipLaunchKernelGGL(k_shade, dim3(blocks_for(cap_rays, 2048)), dim3(kBlock), 0, s, f, it);
    return hipGetLastError();
}

// Free-flight lengths of the path tracer for given random words.
__global__ void k_pt_free_flight(const uint32_t* words, int64_t n, float* out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = pt_free_flight(words[i]);
}

hipError_t launch_pt_free_flight(const uint32_t* words, int64_t n, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pt_free_flight, dim3(blocks_for(n, 4096)), dim3(kBlock), 0, s, words, n, out);
    return hipGetLastError();
}

// A view's per-frame values stored from the launch's arguments (frames that
// use no pinned host block).
__global__ void k_store_var(FrameVar v, FrameVar* dst) {
    if (threadIdx.x == 0) *dst = v;
}

hipError_t launch_store_var(const FrameVar& v, FrameVar* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_store_var, dim3(1), dim3(64), 0, s, v, dst);
    return hipGetLastError();
}

hipError_t launch_frame_end(const FrameDev& f, int max_iters, CacheCtr* cctr, bool reset, const uint32_t* gate,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_frame_end, dim3(1), dim3(64), 0, s, f, max_iters, cctr, reset ? 1 : 0, gate);
    return hipGetLastError();
}

// Pending-ray counts of the first march of up to 64 views, written straight
// into (pinned) host memory: one launch instead of one copy per view.  The
// gate of the frame end is set when none is pending.
struct PendingSrc {
    const uint32_t* p[64];
};

__global__ void k_pending_gather(PendingSrc src, int32_t n, uint32_t* host_out, uint32_t* gate) {
    const int32_t t = threadIdx.x;
    const uint32_t v = t < n ? *src.p[t] : 0u;
    if (t < n) host_out[t] = v;
    const uint64_t any = __ballot(v != 0u);
    if (t == 0) *gate = any == 0ull ? 1u : 0u;
    __threadfence_system();
}

hipError_t launch_pending_gather(const FrameDev* const* fs, int n, int it, uint32_t* host_out, uint32_t* gate,
                                 hipStream_t s) {
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    PendingSrc src{};
    for (int i = 0; i < n; ++i) src.p[i] = &fs[i]->ctr[it].pending;
    hipLaunchKernelGGL(k_pending_gather, dim3(1), dim3(64), 0, s, src, n, host_out, gate);
    return hipGetLastError();
}

}  // namespace cinr
