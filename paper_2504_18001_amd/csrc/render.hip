// Wavefront ray marching through the brick cache (Section 5.1 with the
// sampler of Algorithms 1 and 2 and the fallback of Section 4.3).
//
// One frame is: raygen (box test, compaction of hitting rays in 8x8 pixel
// tiles) -> iterations of { march, infer misses, shade } until no ray is live.
// `march` runs one thread per ray and composites samples as they are served
// by the cache; at the first true miss it switches to gathering a wavefront
// step of S samples (the miss included) into a per-ray buffer, appending
// true-miss records with one atomic per wave.  The INR then infers all misses
// in one batch (Algorithm 1), and `shade` composites the gathered samples in
// order, re-queueing unfinished rays for the next iteration.
#include "frame.h"

namespace cinr {


struct SampleRes {
    int32_t status;
    int32_t slot;
    int64_t req_key;
    float value;
};

// The two most recent page-table lookups of a ray.  Residency is constant
// within a frame, so a repeated key (consecutive samples in the same brick)
// needs no reload.
struct SlotCache {
    int32_t k0 = -1, s0 = -1, k1 = -1, s1 = -1;
    __device__ int32_t lookup(const int32_t* pt, int32_t key) {
        if (key == k0) return s0;
        if (key == k1) {
            const int32_t tk = k0, ts = s0;
            k0 = k1;
            s0 = s1;
            k1 = tk;
            s1 = ts;
            return s0;
        }
        const int32_t v = pt[key];
        k1 = k0;
        s1 = s0;
        k0 = key;
        s0 = v;
        return v;
    }
};

// Sampler of Algorithm 2 for one position: macro-cell skip, stochastic LoD,
// page-table lookup at that LoD and every coarser one, trilinear fetch.
__device__ inline SampleRes sample_cache(const FrameDev& f, const float p[3], SlotCache& sc) {
    SampleRes s;
    s.slot = -1;
    s.req_key = -1;
    s.value = 0.0f;
    if (f.flags) {
        int32_t ci[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ci[a] = (int32_t)fast_div((uint32_t)(int32_t)p[a], f.div_mc);
            if (ci[a] > f.M[a] - 1) ci[a] = f.M[a] - 1;
        }
        if (!f.flags[((int64_t)ci[2] * f.M[1] + ci[1]) * f.M[0] + ci[0]]) {
            s.status = S_SKIP;
            return s;
        }
    }
    s.status = S_MISS;
    if (f.mode != CINR_CACHED) return s;
    const int32_t nl = f.geo.n_lods;
    const int32_t L = select_lod(p, f.cam.eye, f.lod_scale, f.frame_seed, f.lod_floor, nl);
    const int32_t B = f.geo.brick;
    for (int32_t Lp = L; Lp < nl; ++Lp) {
        const BrickAddr a = brick_addr(f.geo, Lp, p);
        if (Lp == L) s.req_key = a.key;
        const int32_t slot = sc.lookup(f.pt, (int32_t)a.key);
        if (slot < 0) continue;
        const float* br = f.pool + (int64_t)slot * (B * B * B) + ((int64_t)a.lj[2] * B + a.lj[1]) * B + a.lj[0];
        const int32_t B2 = B * B;
        const float c000 = br[0], c100 = br[1], c010 = br[B], c110 = br[B + 1];
        const float c001 = br[B2], c101 = br[B2 + 1], c011 = br[B2 + B], c111 = br[B2 + B + 1];
        const float fx = a.frac[0], fy = a.frac[1], fz = a.frac[2];
        const float x00 = __builtin_fmaf(fx, c100 - c000, c000);
        const float x10 = __builtin_fmaf(fx, c110 - c010, c010);
        const float x01 = __builtin_fmaf(fx, c101 - c001, c001);
        const float x11 = __builtin_fmaf(fx, c111 - c011, c011);
        const float y0 = __builtin_fmaf(fy, x10 - x00, x00);
        const float y1 = __builtin_fmaf(fy, x11 - x01, x01);
        s.value = __builtin_fmaf(fz, y1 - y0, y0);
        s.slot = slot;
        s.status = (Lp == L) ? S_HIT : S_FALLBACK;
        break;
    }
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

__device__ inline void flush_requests(const FrameDev& f, int64_t key, uint32_t cnt) {
    if (key < 0 || cnt == 0) return;
    const uint32_t old = atomicAdd(&f.req[key], cnt);
    if (old == 0u) {
        const uint32_t i = atomicAdd(f.n_touched, 1u);
        f.touched[i] = (int32_t)key;
    }
}

__device__ inline void log_miss(const FrameDev& f, int32_t pix, int32_t k, const float p[3]) {
    if (f.misslog_cap <= 0) return;
    const uint32_t i = atomicAdd(f.n_misslog, 1u);
    if ((int32_t)i < f.misslog_cap) {
        MissLogRec r;
        r.pix = pix;
        r.k = k;
        r.x = p[0];
        r.y = p[1];
        r.z = p[2];
        f.misslog[i] = r;
    }
}

struct Tally {
    uint64_t rays = 0, samples = 0, hits = 0, fallbacks = 0, misses = 0, skipped = 0;
    __device__ void add(int32_t st) {
        ++samples;
        hits += st == S_HIT;
        fallbacks += st == S_FALLBACK;
        misses += st == S_MISS;
        skipped += st == S_SKIP;
    }
    // all 64 lanes of the wave must call this together
    __device__ void commit(unsigned long long* stats) {
        wave_add_u64(&stats[ST_RAYS], rays);
        wave_add_u64(&stats[ST_SAMPLES], samples);
        wave_add_u64(&stats[ST_HITS], hits);
        wave_add_u64(&stats[ST_FALLBACKS], fallbacks);
        wave_add_u64(&stats[ST_MISSES], misses);
        wave_add_u64(&stats[ST_SKIPPED], skipped);
    }
};

// Per-ray bookkeeping of one decided sample: request run-length aggregation
// (any sample not served at its own LoD requests its brick) and LRU stamps.
struct RayBook {
    int64_t rk = -1;
    uint32_t rc = 0;
    int32_t last_slot = -1;
    __device__ void note(const FrameDev& f, const SampleRes& s) {
        if (f.mode != CINR_CACHED || s.status == S_SKIP) return;
        if (s.status != S_HIT) {
            if (s.req_key != rk) {
                flush_requests(f, rk, rc);
                rk = s.req_key;
                rc = 1;
            } else {
                ++rc;
            }
        }
        if (s.slot >= 0 && s.slot != last_slot) {
            // many rays stamp the same slot: store only if not yet stamped in
            // this frame, so that the L2 does not serialise identical stores
            if (f.last_used[s.slot] != f.frame) f.last_used[s.slot] = f.frame;
            last_slot = s.slot;
        }
    }
    __device__ void flush(const FrameDev& f) {
        flush_requests(f, rk, rc);
        rk = -1;
        rc = 0;
    }
};

__global__ __launch_bounds__(kBlock) void k_frame_begin(FrameDev f, int32_t n_ctr, uint8_t* flags,
                                                        const float* minmax, int64_t n_cells, CacheCtr* cctr) {
    __shared__ float alpha[256];
    alpha[threadIdx.x] = f.tf[4 * threadIdx.x + 3];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n_ctr) f.ctr[t] = IterCtr{0u, 0u, 0u, 0u};
    if (t < ST_COUNT) f.stats[t] = 0ull;
    if (t == 0 && cctr) cctr->n_misslog = 0u;
    // macro-cell flags (Section 5.2): maximum opacity over the TF rows a
    // cell's value range can reach; zero means the cell is skipped
    if (flags && t < n_cells) {
        const float a = minmax[2 * t] * 255.0f;
        const float b = minmax[2 * t + 1] * 255.0f;
        int32_t lo = (int32_t)__builtin_floorf(a), hi = (int32_t)__builtin_ceilf(b);
        lo = lo < 0 ? 0 : lo;
        hi = hi > 255 ? 255 : hi;
        float mu = 0.0f;
        for (int32_t r = lo; r <= hi; ++r) mu = alpha[r] > mu ? alpha[r] : mu;
        flags[t] = mu > 0.0f ? 1 : 0;
    }
}

// One thread per ray.  Iteration 0 walks all pixels in 8x8 tiles (one tile
// per wave) and generates the rays itself; later iterations walk the list
// of rays re-queued by k_shade.  Every lane of a wave runs the same number
// of loop trips so that list reservations can be made per wave.
template <int kPipe>
__global__ __launch_bounds__(kBlock) void k_march(FrameDev f, int32_t it, uint32_t n0) {
    __shared__ float4 tfs[256];
    tfs[threadIdx.x] = reinterpret_cast<const float4*>(f.tf)[threadIdx.x];
    __syncthreads();
    const uint32_t n = it == 0 ? n0 : f.ctr[it].live;
    const int32_t* cur = (it & 1) ? f.live1 : f.live0;
    // The ray list is cut into 8*bands contiguous bands; XCD x (workgroups are
    // dispatched round-robin over the 8 XCDs) walks bands x, x+8, ...  Each
    // band is a compact image region (locality in one XCD's L2) and every XCD
    // gets bands from all over the image (balance).
    const uint32_t nb = gridDim.x;
    const uint32_t bands = (uint32_t)f.xcd_bands;
    const uint32_t bs = nb / (8u * bands);  // workgroups per band
    const uint32_t x = blockIdx.x & 7u, i8 = blockIdx.x >> 3;
    const uint32_t lb = (x + 8u * (i8 / bs)) * bs + (i8 % bs);
    const uint32_t per = (n + nb - 1) / nb;
    const uint32_t beg = lb * per;
    const uint32_t end = beg + per < n ? beg + per : n;
    const int32_t tiles_x = (f.cam.W + 7) / 8;
    Tally tally;
    const int32_t S = f.S;
    for (uint32_t r0 = beg; r0 < end; r0 += kBlock) {
        const uint32_t r = r0 + threadIdx.x;
        bool has = r < end;
        int32_t pix = 0;
        float o[3], d[3], ts = 0.0f, te = -1.0f;
        if (has) {
            int32_t i, j;
            if (it == 0) {
                const uint32_t tile = r >> 6, w = r & 63u;
                i = (int32_t)(tile % (uint32_t)tiles_x) * 8 + (int32_t)(w & 7u);
                j = (int32_t)(tile / (uint32_t)tiles_x) * 8 + (int32_t)(w >> 3);
                has = i < f.cam.W && j < f.cam.H;
            } else {
                pix = cur[r];
                i = pix % f.cam.W;
                j = pix / f.cam.W;
            }
            if (has) {
                if (it == 0) pix = j * f.cam.W + i;
                const bool hit = ray_setup(f.cam, f.vm1, i, j, o, d, ts, te);
                if (it == 0) {
                    if (!hit) f.rgba[pix] = make_float4(0.f, 0.f, 0.f, 0.f);
                    tally.rays += hit;
                }
                has = hit;
            }
        }
        int32_t k = 0;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        if (has && it > 0) {
            k = f.k_next[pix];
            acc = f.rgba[pix];
        }
        RayBook book;
        SlotCache sc;
        bool pend = false;
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
                        grp[u] = sample_cache(f, p, sc);
                        ++cnt;
                    }
                }
                if (cnt < kPipe) run = false;
#pragma unroll
                for (int u = 0; u < kPipe; ++u) {
                    if (u >= cnt) break;
                    const SampleRes& sr = grp[u];
                    tally.add(sr.status);
                    book.note(f, sr);
                    if (sr.status == S_MISS) {
                        pend = true;
                        run = false;
                        break;
                    }
                    if (sr.status != S_SKIP) composite(acc, sr.value, tfs, f.step);
                    ++k;
                    if (f.ert_on && acc.w >= f.ert) {
                        run = false;
                        break;
                    }
                }
            }
        }
        // a wavefront step of S samples starting at the miss
        const uint32_t pi = wave_reserve(pend ? 1u : 0u, &f.ctr[it].pending);
        uint64_t mask = 0;
        int32_t nc = 0;
        if (pend) {
            f.pend_pix[pi] = pix;
            float* vb = f.vals + (int64_t)pi * S;
            mask = 1;
            nc = 1;
            while (nc < S) {
                float q[3];
                if (!sample_pos(o, d, ts, te, f.step, k + nc, f.vm1, q)) break;
                const SampleRes sr = sample_cache(f, q, sc);
                tally.add(sr.status);
                book.note(f, sr);
                if (sr.status == S_MISS)
                    mask |= 1ull << nc;
                else
                    vb[nc] = sr.status == S_SKIP ? -1.0f : sr.value;
                ++nc;
            }
            f.pend_n[pi] = nc;
            f.k_next[pix] = k;
        }
        // true-miss records (position, destination slot), reserved per wave
        uint32_t mb = wave_reserve((uint32_t)__popcll(mask), &f.ctr[it].misses);
        if (pend) {
            for (int32_t sidx = 0; sidx < nc; ++sidx) {
                if (!((mask >> sidx) & 1ull)) continue;
                float q[3];
                sample_pos(o, d, ts, te, f.step, k + sidx, f.vm1, q);
                f.miss_rec[mb++] = make_float4(q[0], q[1], q[2], __uint_as_float(pi * (uint32_t)S + (uint32_t)sidx));
                log_miss(f, pix, k + sidx, q);
            }
        }
        if (has) {
            book.flush(f);
            f.rgba[pix] = acc;
        }
    }
    tally.commit(f.stats);
}

__global__ __launch_bounds__(kBlock) void k_shade(FrameDev f, int32_t it) {
    __shared__ float4 tfs[256];
    tfs[threadIdx.x] = reinterpret_cast<const float4*>(f.tf)[threadIdx.x];
    __syncthreads();
    const uint32_t n = f.ctr[it].pending;
    int32_t* next = (it & 1) ? f.live0 : f.live1;
    const int32_t S = f.S;
    for (uint32_t pi = blockIdx.x * kBlock + threadIdx.x; pi < n; pi += gridDim.x * kBlock) {
        const int32_t pix = f.pend_pix[pi];
        const int32_t nc = f.pend_n[pi];
        int32_t k = f.k_next[pix];
        float4 acc = f.rgba[pix];
        const float* vb = f.vals + (int64_t)pi * S;
        bool done = false;
        for (int32_t s = 0; s < nc; ++s) {
            const float v = vb[s];
            if (v >= 0.0f) composite(acc, v, tfs, f.step);
            if (f.ert_on && acc.w >= f.ert) {
                done = true;
                break;
            }
        }
        if (!done) {
            k += nc;
            const int32_t i = pix % f.cam.W, j = pix / f.cam.W;
            float o[3], d[3], ts, te;
            ray_setup(f.cam, f.vm1, i, j, o, d, ts, te);
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

__global__ void k_frame_end(FrameDev f, int32_t n_iters, CacheCtr* cctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        f.stats[ST_ITERS] = (unsigned long long)n_iters;
        if (cctr) {
            f.stats[ST_REQUESTED] = cctr->n_touched;
            f.stats[ST_SELECTED] = cctr->n_sel;
            f.stats[ST_EVICTED] = cctr->need_evict;
            cctr->n_touched = 0u;  // the next frame's requests start empty
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

hipError_t launch_frame_begin(const FrameDev& f, int32_t n_iter_ctr, const uint8_t* flags_out, const float* minmax,
                              int64_t n_cells, CacheCtr* cctr, hipStream_t s) {
    int64_t n = n_iter_ctr;
    if (flags_out && n_cells > n) n = n_cells;
    if (n < ST_COUNT) n = ST_COUNT;
    hipLaunchKernelGGL(k_frame_begin, dim3(blocks_for(n, 1 << 20)), dim3(kBlock), 0, s, f, n_iter_ctr,
                       (uint8_t*)flags_out, minmax, flags_out ? n_cells : 0, cctr);
    return hipGetLastError();
}

hipError_t launch_march(const FrameDev& f, int it, int64_t cap_rays, hipStream_t s) {
    // iteration 0 walks all pixels in 8x8 tiles, one workgroup per 256 pixels
    const uint32_t n0 = (uint32_t)(((f.cam.W + 7) / 8) * ((f.cam.H + 7) / 8)) * 64u;
    const int64_t cap = it == 0 ? (int64_t)n0 : cap_rays;
    // a multiple of 8 * bands workgroups
    const int64_t q = 8LL * f.xcd_bands;
    int64_t b = (cap + kBlock - 1) / kBlock;
    b = b > (1 << 20) ? (1 << 20) : b;
    b = ((b + q - 1) / q) * q;
    // kPipe: samples decided and fetched ahead in the fast phase
    switch (f.pipe) {
        case 1: hipLaunchKernelGGL(k_march<1>, dim3((unsigned)b), dim3(kBlock), 0, s, f, it, n0); break;
        case 2: hipLaunchKernelGGL(k_march<2>, dim3((unsigned)b), dim3(kBlock), 0, s, f, it, n0); break;
        case 8: hipLaunchKernelGGL(k_march<8>, dim3((unsigned)b), dim3(kBlock), 0, s, f, it, n0); break;
        default: hipLaunchKernelGGL(k_march<4>, dim3((unsigned)b), dim3(kBlock), 0, s, f, it, n0); break;
    }
    return hipGetLastError();
}

hipError_t launch_shade(const FrameDev& f, int it, int64_t cap_rays, hipStream_t s) {
    hipLaunchKernelGGL(k_shade, dim3(blocks_for(cap_rays, 2048)), dim3(kBlock), 0, s, f, it);
    return hipGetLastError();
}

hipError_t launch_frame_end(const FrameDev& f, int n_iters, CacheCtr* cctr, hipStream_t s) {
    hipLaunchKernelGGL(k_frame_end, dim3(1), dim3(64), 0, s, f, n_iters, cctr);
    return hipGetLastError();
}

}  // namespace cinr
