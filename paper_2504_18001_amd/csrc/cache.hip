// Cache manager and request handler of Section 4.3 on the GPU.
//
// End of frame f:
//  rank     over the bricks requested in f (the "touched" list built by the
//           sampler): rank = f + c - 1 when first seen, else rank + c, clamped
//           to f + window (Section 4.3.3); each gets a 64-bit score
//           (rank << 32 | ~key) -- or ~key for key order -- so that the
//           request list is the set of largest scores, ties broken by key.
//  top-k    tournament selection: each workgroup sorts 2048 scores in LDS
//           (bitonic) and keeps its best k; repeated until one workgroup is
//           left.  Deterministic: scores are unique.
//  insert   lowest free slots first (free slots are always the tail
//           [n_used, pool)), then the least recently used slots by
//           (last_used, slot) -- the same top-k on ~(last_used << 32 | slot).
//           Evicted bricks are unmapped and their ranks forgotten; new bricks
//           are mapped and stamped f + 1, then decoded into their slots.
//  The frame index f is read from the cache counters (set by the frame's
//  first k_frame_begin), so that these launches can be replayed unchanged.
#include "frame.h"

namespace cinr {

__global__ void k_cache_init(CacheDev c, int64_t n_keys, int64_t n_dir) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_keys; t += stride) {
        if (c.pt) c.pt[t] = -1;
        c.rank[t] = -1;
        c.req[t] = 0u;
        if (c.last_req) c.last_req[t] = 0u;
    }
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < c.pool_bricks; t += stride) {
        c.owner[t] = -1;
        c.last_used[t] = -1;
    }
    if (c.vdir) {
        // two-level page table: no block in use, every block entry unmapped,
        // the free stack pops blocks 0, 1, 2, ... first
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_dir; t += stride) c.vdir[t] = -1;
        const int64_t ne = (int64_t)c.vcap * kVptEntries;
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ne; t += stride) c.vblk[t] = -1;
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < c.vcap; t += stride) {
            c.vcnt[t] = 0;
            c.vfree[t] = c.vcap - 1 - (int32_t)t;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *c.ctr = CacheCtr{};
        c.ctr->v_free = (uint32_t)c.vcap;
    }
}

// Clears the request counts kept for dumps (before the frame's sampler).
__global__ void k_clear_last_req(CacheDev c, int64_t n_keys) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_keys; t += (int64_t)gridDim.x * blockDim.x)
        c.last_req[t] = 0u;
}

// Scores of the touched bricks base + e, e = threadIdx.x + 256 q < have,
// after their rank update (first selection pass), into s[e]; s[e] = 0 for
// have <= e < m.  Each thread's keys are read together, then their counts
// and ranks, so that a thread waits for three round trips in all rather
// than three per brick (the touched keys are distinct: no two threads write
// the same entries).
__device__ inline void rank_scores(const RankArgs& ra, int32_t frame, uint64_t base, uint32_t have, uint32_t m,
                                   uint64_t* s) {
    constexpr int kPer = kTopkChunk / 256;
    int32_t key[kPer];
    uint32_t cnt[kPer];
    int64_t old[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t e = threadIdx.x + 256u * q;
        key[q] = e < have ? ra.touched[base + e] : -1;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        cnt[q] = key[q] >= 0 ? ra.req[key[q]] : 0u;
        old[q] = key[q] >= 0 ? ra.rank[key[q]] : 0;
    }
    const int64_t cap = (int64_t)frame + ra.window;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t e = threadIdx.x + 256u * q;
        if (e >= m) continue;
        if (key[q] < 0) {
            s[e] = 0ull;
            continue;
        }
        int64_t r = old[q] < 0 ? (int64_t)frame + (int64_t)cnt[q] - 1 : old[q] + (int64_t)cnt[q];
        if (r > cap) r = cap;
        if (ra.last_req) ra.last_req[key[q]] = cnt[q];
        ra.rank[key[q]] = r;
        ra.req[key[q]] = 0u;
        const uint64_t low = 0xFFFFFFFFull - (uint64_t)(uint32_t)key[q];
        s[e] = ra.ranking ? (((uint64_t)r << 32) | low) : low;
    }
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, uint32_t mask) {
    const uint32_t lo = __shfl_xor((uint32_t)v, (int)mask);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), (int)mask);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of s[0, 256 E) in descending order with E elements per thread
// in registers (thread t holds elements t E .. t E + E - 1): the steps whose
// partner is in the same thread compare in registers, those whose partner
// thread is in the same wavefront exchange by shuffles, and only the steps
// across wavefronts go through LDS.  The same network as sort_desc.
template <int E>
__device__ void sort_desc_regs(uint64_t* s) {
    constexpr uint32_t m = 256u * E;
    const uint32_t t = threadIdx.x;
    uint64_t v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = s[t * E + q];
    for (uint32_t len = 2; len <= m; len <<= 1) {
        // partners in other threads: element t E + q pairs with (t ^ pt) E + q
        for (uint32_t j = len >> 1; j >= (uint32_t)E; j >>= 1) {
            const uint32_t pt = j / E;
            uint64_t o[E];
            if (pt < 64u) {
#pragma unroll
                for (int q = 0; q < E; ++q) o[q] = shfl_xor_u64(v[q], pt);
            } else {
                __syncthreads();  // the previous exchange's reads are done
#pragma unroll
                for (int q = 0; q < E; ++q) s[t * E + q] = v[q];
                __syncthreads();
#pragma unroll
                for (int q = 0; q < E; ++q) o[q] = s[(t ^ pt) * E + q];
            }
            const bool lower = (t & pt) == 0u;
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const bool desc = ((t * E + q) & len) == 0u;
                const uint64_t hi = v[q] > o[q] ? v[q] : o[q];
                const uint64_t lo = v[q] > o[q] ? o[q] : v[q];
                v[q] = (lower == desc) ? hi : lo;
            }
        }
        // partners in the same thread (compile-time indices: registers)
#pragma unroll
        for (int jj = E / 2; jj >= 1; jj >>= 1) {
            if ((uint32_t)jj >= len) continue;
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int x = q ^ jj;
                if (x > q) {
                    const bool desc = ((t * E + q) & len) == 0u;
                    const uint64_t a = v[q], b = v[x];
                    if (desc ? (a < b) : (a > b)) {
                        v[q] = b;
                        v[x] = a;
                    }
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E; ++q) s[t * E + q] = v[q];
    __syncthreads();
}

// Bitonic sort of s[0, m) in descending order (m a power of two, <= 2048),
// by the 256 threads of the workgroup.
__device__ void sort_desc(uint64_t* s, uint32_t m) {
    switch (m) {
        case 256: sort_desc_regs<1>(s); return;
        case 512: sort_desc_regs<2>(s); return;
        case 1024: sort_desc_regs<4>(s); return;
        case 2048: sort_desc_regs<8>(s); return;
        default: break;
    }
    for (uint32_t len = 2; len <= m; len <<= 1) {
        for (uint32_t j = len >> 1; j > 0; j >>= 1) {
            for (uint32_t e = threadIdx.x; e < m; e += 256) {
                const uint32_t x = e ^ j;
                if (x > e) {
                    const uint64_t p = s[e], q = s[x];
                    const bool desc = (e & len) == 0;
                    if (desc ? (p < q) : (p > q)) {
                        s[e] = q;
                        s[x] = p;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// LoD of a key of any of the cache's volumes.
__device__ inline int32_t key_lod(const CacheGeom& g, int64_t key) {
    const int64_t k = key % g.keys_per_vol;
    int32_t L = 0;
    while (L + 1 < g.n_lods && k >= g.lod[L + 1].off) ++L;
    return L;
}

// Slot class of a key: 1 for the binary16 class of a mixed pool, else 0.
__device__ inline uint32_t key_class(const CacheDev& c, const CacheGeom& g, int32_t key) {
    if (c.pool_kind != POOL_MIXED || key < 0 || (int64_t)key >= g.n_keys) return 0u;
    return (c.f16_lods >> key_lod(g, key)) & 1u;
}

// Exclusive count of `pred` over the lower threads of a 256-thread
// workgroup (4 wavefronts of 64), and the workgroup's total; every thread
// calls it.  wc: 4 words of LDS.
__device__ inline uint32_t block_prefix(bool pred, uint32_t* total, uint32_t* wc) {
    const unsigned long long m = __ballot(pred);
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    if (lane == 0u) wc[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = (uint32_t)__popcll(m & ((1ull << lane) - 1ull)), tot = 0u;
    for (uint32_t k = 0; k < 4u; ++k) {
        if (k < w) before += wc[k];
        tot += wc[k];
    }
    __syncthreads();  // wc is reused by the next call
    *total = tot;
    return before;
}

__device__ inline uint32_t pow2_at_least(uint32_t n) {
    uint32_t m = 1;
    while (m < n) m <<= 1;
    return m;
}

// Insertion of the selected bricks [t0, n_sel) step `stride` (Section 4.3.1):
// the lowest free slots first, then the LRU victims, within the slot class
// of each brick; evicted bricks are unmapped and their ranks forgotten, new
// bricks are mapped, stamped and queued for decoding.  `ctr` is the
// counters' state after the selection; ins_slots holds each entry's rank
// among the entries of its class (overwritten with the slot).
__device__ void insert_entries(const CacheDev& c, const CacheGeom& g, const CacheCtr& ctr, uint32_t t0,
                               uint32_t stride) {
    const int32_t stamp = ctr.frame + 1;
    for (uint32_t t = t0; t < ctr.n_sel; t += stride) {
        const int32_t key = c.ins_keys[t];
        const uint32_t cl = key_class(c, g, key);
        const uint32_t r = (uint32_t)c.ins_slots[t];
        const uint32_t n_free = cl ? ctr.n_free1 : ctr.n_free;
        int32_t slot;
        if (r < n_free)
            slot = (int32_t)((cl ? (uint32_t)c.split + ctr.n_used1 : ctr.n_used) + r);
        else
            slot = (int32_t)(uint32_t)(~(cl ? c.vic1 : c.vic)[r - n_free] & 0xFFFFFFFFull);
        bool ok = key >= 0 && (int64_t)key < g.n_keys && slot >= 0 && slot < c.pool_bricks;
        int32_t old = -1;
        if (ok) {
            old = c.owner[slot];
            if (old >= 0) {
                if (c.pt) c.pt[old] = -1;
                c.rank[old] = -1;
            }
            if (c.pt) c.pt[key] = slot;  // a two-level table is updated by k_vpt_update
            c.owner[slot] = key;
            c.last_used[slot] = stamp;
        }
        c.ins_old[t] = old;
        // volume and brick coordinates of the key
        const int32_t vol = ok ? (int32_t)((int64_t)key / g.keys_per_vol) : 0;
        const int64_t vkey = ok ? (int64_t)key - (int64_t)vol * g.keys_per_vol : 0;
        int32_t L = 0;
        while (L + 1 < g.n_lods && vkey >= g.lod[L + 1].off) ++L;
        const int64_t local = vkey - g.lod[L].off;
        c.ins_vols[t] = vol;
        const int32_t nbx = g.lod[L].nb[0], nby = g.lod[L].nb[1];
        c.ins_slots[t] = ok ? slot : -1;  // an invalid entry is not decoded
        int32_t* q = c.ins_reqs + 4 * (int64_t)t;
        q[0] = ok ? L : -1;
        q[1] = (int32_t)(local % nbx);
        q[2] = (int32_t)((local / nbx) % nby);
        q[3] = (int32_t)(local / ((int64_t)nbx * nby));
        const uint32_t e = ctr.n_evlog + t;
        if (ok && (int32_t)e < c.evlog_cap) {
            int32_t* r = c.evlog + 4 * (int64_t)e;
            r[0] = stamp;
            r[1] = slot;
            r[2] = old;
            r[3] = key;
        }
    }
}

// Occupancy and eviction-log counters after an insertion (one thread).
__device__ inline void insert_counters(CacheCtr* out, const CacheCtr& ctr) {
    const uint32_t n0 = ctr.n_sel - ctr.n_sel1;
    out->n_used = ctr.n_used + (n0 < ctr.n_free ? n0 : ctr.n_free);
    out->n_used1 = ctr.n_used1 + (ctr.n_sel1 < ctr.n_free1 ? ctr.n_sel1 : ctr.n_free1);
    out->n_evlog = ctr.n_evlog + ctr.n_sel;
}

// Frame statistics of the views of the frame (one thread): iterations from
// each view's per-iteration counters (launches 0 .. n-1, where n - 1 is the
// first iteration that left no ray pending, or max_iters - 1), the cache
// manager's counters of the whole frame.  Clears the request list.
__device__ void views_frame_stats(const CacheDev& c, uint32_t n_touched, uint32_t n_sel, uint32_t need_evict) {
    const uint32_t nv = c.ctr->n_views < (uint32_t)kMaxFrameViews ? c.ctr->n_views : (uint32_t)kMaxFrameViews;
    for (uint32_t v = 0; v < nv; ++v) {
        const ViewEnd e = c.views[v];
        int32_t n = 1;
        while (n < e.max_iters && e.ctr[n - 1].pending != 0u) ++n;
        e.stats[ST_ITERS] = (unsigned long long)n;
        e.stats[ST_REQUESTED] = n_touched;
        e.stats[ST_SELECTED] = n_sel;
        e.stats[ST_EVICTED] = need_evict;
    }
    c.ctr->n_touched = 0u;  // the next frame's requests start empty
}

// One tournament pass: workgroup b sorts its elements [b*2048, (b+1)*2048)
// of the pass input in descending order and writes the best k to
// out[b*k ...].  The number of live input elements of pass p follows from
// the device count of pass 0 (each pass keeps k per 2048), so empty
// workgroups skip the sort and partial ones sort only a power of two
// covering their elements.  Sources of pass 0: a score array, the LRU order
// of the slots [0, count) scored ~(last_used << 32 | slot), or the touched
// bricks ranked on the fly.  The final pass may also publish the request
// list (select epilogue), then insert the selected bricks and write the
// views' frame statistics (tail).  A fused launch is pass 0 followed, in
// the last of its workgroups to finish, by pass 1 (two-pass selections).
__global__ __launch_bounds__(256) void k_topk(TopkArgs a) {
    __shared__ uint64_t s[kTopkChunk];
    __shared__ uint32_t nsel, ticket, wc[4];
    if (a.gate && *a.gate == 0u) return;
    if (a.frame_gate && *a.frame_gate == 0u) return;
    uint64_t c = a.cap0;
    if (a.count_dev && (uint64_t)*a.count_dev < c) c = *a.count_dev;
    const uint64_t n_touched = c;
    // every live element in pass 0's first workgroup: it sorts them all and
    // completes the selection; the later passes have nothing to do
    const bool one = n_touched <= (uint64_t)kTopkChunk;
    if (one && a.pass > 0) return;
    const bool last = one || (!a.fused && a.pass == a.last_pass);
    if (!one)
        for (int q = 0; q < a.pass; ++q) c = ((c + kTopkChunk - 1) / kTopkChunk) * (uint64_t)a.k;
    const uint64_t base = (uint64_t)blockIdx.x * kTopkChunk;
    if (base >= c && blockIdx.x > 0 && (one || !a.fused)) return;
    const uint32_t have = base >= c ? 0u : (uint32_t)(c - base < kTopkChunk ? c - base : kTopkChunk);
    uint32_t m = pow2_at_least(have);
    if (have > 0 || blockIdx.x == 0) {
        if (a.pass == 0 && a.mode == TOPK_RANK) {
            rank_scores(a.ra, *a.ra.frame, base, have, m, s);
        } else {
            for (uint32_t e = threadIdx.x; e < m; e += 256) {
                const uint64_t idx = base + e;
                uint64_t v = 0ull;
                if (e < have) {
                    if (a.pass == 0 && a.mode == TOPK_LRU) {
                        const uint64_t slot = idx + (uint64_t)a.lru_base;
                        v = ~(((uint64_t)(uint32_t)a.lru_last_used[slot] << 32) | slot);
                    } else {
                        v = a.in[idx];
                    }
                }
                s[e] = v;
            }
        }
        __syncthreads();
        sort_desc(s, m);
        uint64_t* out = last ? a.final_out : a.out + (uint64_t)blockIdx.x * a.k;
        for (int32_t e = threadIdx.x; e < a.k; e += 256) out[e] = (uint32_t)e < m ? s[e] : 0ull;
    }
    if (a.fused && !one) {
        // the last workgroup to finish pass 0 runs the later passes, chunk by
        // chunk, ping-ponging between out and out2, the last into final_out
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) ticket = atomicAdd(a.done, 1u);
        __syncthreads();
        if (ticket != gridDim.x - 1u) return;
        __threadfence();
        if (threadIdx.x == 0) *a.done = 0u;
        uint64_t cc = ((c + kTopkChunk - 1) / kTopkChunk) * (uint64_t)a.k;  // live elements of pass 1
        const uint64_t* src = a.out;
        for (int p = 1; cc > (uint64_t)kTopkChunk; ++p) {
            uint64_t* dst = (p & 1) ? a.out2 : a.out;
            const uint64_t nb = (cc + kTopkChunk - 1) / kTopkChunk;
            for (uint64_t b = 0; b < nb; ++b) {
                const uint64_t rest = cc - b * kTopkChunk;
                const uint32_t h = (uint32_t)(rest < kTopkChunk ? rest : kTopkChunk);
                m = pow2_at_least(h);
                __syncthreads();
                for (uint32_t e = threadIdx.x; e < m; e += 256) s[e] = e < h ? src[b * kTopkChunk + e] : 0ull;
                __syncthreads();
                sort_desc(s, m);
                for (int32_t e = threadIdx.x; e < a.k; e += 256) dst[b * a.k + e] = (uint32_t)e < m ? s[e] : 0ull;
            }
            __threadfence();
            __syncthreads();
            src = dst;
            cc = nb * (uint64_t)a.k;
        }
        const uint32_t h = (uint32_t)cc;
        m = pow2_at_least(h);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < m; e += 256) s[e] = e < h ? src[e] : 0ull;
        __syncthreads();
        sort_desc(s, m);
        for (int32_t e = threadIdx.x; e < a.k; e += 256) a.final_out[e] = (uint32_t)e < m ? s[e] : 0ull;
    }
    if (a.sel.ctr && (last || a.fused)) {
        // request list: keys of the non-zero scores, best first
        if (threadIdx.x == 0) nsel = 0u;
        __syncthreads();
        for (int32_t t = threadIdx.x; t < a.sel.lim; t += 256) {
            const uint64_t v = (uint32_t)t < m ? s[t] : 0ull;
            if (v != 0ull) {
                a.sel.ins_keys[t] = (int32_t)(0xFFFFFFFFull - (v & 0xFFFFFFFFull));
                atomicAdd(&nsel, 1u);
            }
        }
        __syncthreads();
        // each entry's rank within its slot class (the selection is at most
        // 256 bricks: one entry per thread)
        const CacheDev& cd = a.tail.c;
        const uint32_t t = threadIdx.x;
        const uint32_t cl = t < nsel ? key_class(cd, a.tail.g, a.sel.ins_keys[t]) : 0u;
        uint32_t n1;
        const uint32_t r1 = block_prefix(cl != 0u, &n1, wc);
        if (t < nsel) cd.ins_slots[t] = (int32_t)(cl ? r1 : t - r1);
        CacheCtr* ctr = a.sel.ctr;
        const uint32_t n_free = (uint32_t)cd.split - ctr->n_used;
        const uint32_t n_free1 = (uint32_t)(cd.pool_bricks - cd.split) - ctr->n_used1;
        const uint32_t need_evict = nsel - n1 > n_free ? nsel - n1 - n_free : 0u;
        const uint32_t need_evict1 = n1 > n_free1 ? n1 - n_free1 : 0u;
        CacheCtr snap = *ctr;
        snap.n_sel = nsel;
        snap.n_free = n_free;
        snap.need_evict = need_evict;
        snap.n_sel1 = n1;
        snap.n_free1 = n_free1;
        snap.need_evict1 = need_evict1;
        __syncthreads();
        if (threadIdx.x == 0) {
            ctr->n_sel = nsel;
            ctr->n_free = n_free;
            ctr->need_evict = need_evict;
            ctr->n_sel1 = n1;
            ctr->n_free1 = n_free1;
            ctr->need_evict1 = need_evict1;
        }
        if (a.tail.insert) {
            insert_entries(cd, a.tail.g, snap, threadIdx.x, 256u);
            __syncthreads();
            if (threadIdx.x == 0) insert_counters(ctr, snap);
        }
        if (a.tail.stats && threadIdx.x == 0)
            views_frame_stats(cd, (uint32_t)n_touched, nsel, need_evict + need_evict1);
    }
}

// Prefill (one workgroup): the given keys are inserted into free slots of
// their class only; the keys that find one are listed in order, with their
// rank in the class, and the others dropped (error bit 1).
__global__ __launch_bounds__(256) void k_prefill_setup(CacheDev c, CacheGeom g, const int32_t* keys, int32_t n,
                                                       int32_t stamp) {
    __shared__ uint32_t wc[4];
    CacheCtr* ctr = c.ctr;
    const uint32_t n_free = (uint32_t)c.split - ctr->n_used;
    const uint32_t n_free1 = (uint32_t)(c.pool_bricks - c.split) - ctr->n_used1;
    uint32_t seen1 = 0u, kept = 0u, kept1 = 0u;
    for (int32_t base = 0; base < n; base += 256) {
        const int32_t t = base + (int32_t)threadIdx.x;
        const bool in = t < n;
        const int32_t key = in ? keys[t] : -1;
        const uint32_t cl = in ? key_class(c, g, key) : 0u;
        uint32_t tot1, tot_kept, tot_kept1;
        const uint32_t r1 = seen1 + block_prefix(in && cl != 0u, &tot1, wc);
        const uint32_t r = cl ? r1 : (uint32_t)t - r1;
        const bool fit = in && r < (cl ? n_free1 : n_free);
        const uint32_t pos = kept + block_prefix(fit, &tot_kept, wc);
        block_prefix(fit && cl != 0u, &tot_kept1, wc);
        if (fit) {
            c.ins_keys[pos] = key;
            c.ins_slots[pos] = (int32_t)r;
        }
        seen1 += tot1;
        kept += tot_kept;
        kept1 += tot_kept1;
    }
    if (threadIdx.x == 0) {
        if (kept < (uint32_t)n) ctr->error |= 1u;
        ctr->frame = stamp - 1;  // k_insert stamps frame + 1
        ctr->n_sel = kept;
        ctr->n_free = n_free;
        ctr->need_evict = 0u;
        ctr->n_sel1 = kept1;
        ctr->n_free1 = n_free1;
        ctr->need_evict1 = 0u;
    }
}

__global__ void k_insert(CacheDev c, CacheGeom g, int32_t finish_inline, const uint32_t* gate) {
    if (gate && *gate == 0u) return;
    const CacheCtr ctr = *c.ctr;
    insert_entries(c, g, ctr, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
    if (finish_inline) {  // single-workgroup launch: update the counters here
        __syncthreads();
        if (threadIdx.x == 0) insert_counters(c.ctr, ctr);
    }
}

__global__ void k_insert_finish(CacheDev c, const uint32_t* gate) {
    if (gate && *gate == 0u) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const CacheCtr ctr = *c.ctr;
        insert_counters(c.ctr, ctr);
    }
}

// Two-level page table after an insertion batch (Section 4.3.1's
// virtualised page tables), one workgroup: unmap the evicted bricks, return
// the blocks they leave empty to the free stack, take a block for each
// directory entry a new brick needs, map the new bricks.  A block returns to
// the stack only once all of its entries are -1 again, so a block taken from
// the stack needs no clearing.  Which block serves a directory entry depends
// on the order of the atomics; the mapping itself (brick -> slot) does not.
constexpr int32_t kVptClaim = -2;  // directory entry being given a block

// Directory and count words change under atomics within k_vpt_update: read
// them at device scope (past the workgroup's L1).
__device__ inline int32_t vpt_load(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(1024) void k_vpt_update(CacheDev c, CacheGeom g, const uint32_t* gate) {
    if (gate && *gate == 0u) return;
    __shared__ uint32_t top, fail;
    const uint32_t n = c.ctr->n_sel;
    if (threadIdx.x == 0) {
        top = c.ctr->v_free;
        fail = 0u;
    }
    for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) {
        const int32_t old = c.ins_old[t];
        if (old < 0) continue;
        int64_t d;
        int32_t e;
        vpt_addr(g, old, &d, &e);
        const int32_t b = vpt_load(&c.vdir[d]);
        if (b < 0) continue;
        const int64_t ix = (int64_t)b * kVptEntries + e;
        if (c.vblk[ix] < 0) continue;  // left unmapped for want of a block
        c.vblk[ix] = -1;
        atomicSub(&c.vcnt[b], 1);
    }
    __threadfence();
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) {
        const int32_t old = c.ins_old[t];
        if (old < 0) continue;
        int64_t d;
        int32_t e;
        vpt_addr(g, old, &d, &e);
        const int32_t b = vpt_load(&c.vdir[d]);
        if (b >= 0 && vpt_load(&c.vcnt[b]) == 0 && atomicCAS(&c.vdir[d], b, -1) == b) c.vfree[atomicAdd(&top, 1u)] = b;
    }
    __threadfence();
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) {
        if (c.ins_slots[t] < 0) continue;
        int64_t d;
        int32_t e;
        vpt_addr(g, c.ins_keys[t], &d, &e);
        if (vpt_load(&c.vdir[d]) != -1 || atomicCAS(&c.vdir[d], -1, kVptClaim) != -1) continue;
        const uint32_t i = atomicSub(&top, 1u);
        if ((int32_t)i <= 0) {
            atomicExch(&c.vdir[d], -1);  // no block left (the pool of blocks was sized below its bound)
        } else {
            atomicExch(&c.vdir[d], vpt_load(&c.vfree[i - 1u]));
        }
    }
    __threadfence();
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) {
        const int32_t slot = c.ins_slots[t];
        if (slot < 0) continue;
        int64_t d;
        int32_t e;
        vpt_addr(g, c.ins_keys[t], &d, &e);
        const int32_t b = vpt_load(&c.vdir[d]);
        if (b < 0) {
            atomicAdd(&fail, 1u);  // the brick stays unmapped
            continue;
        }
        c.vblk[(int64_t)b * kVptEntries + e] = slot;
        atomicAdd(&c.vcnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c.ctr->v_free = (int32_t)top < 0 ? 0u : top;
        c.ctr->v_fail += fail;
    }
}

// ---------------------------------------------------------------------------

hipError_t launch_cache_init(const CacheDev& c, int64_t n_keys, int64_t n_dir, hipStream_t s) {
    int64_t n = n_keys > c.pool_bricks ? n_keys : c.pool_bricks;
    if (c.vdir) {
        n = n > n_dir ? n : n_dir;
        n = n > (int64_t)c.vcap * kVptEntries ? n : (int64_t)c.vcap * kVptEntries;
    }
    int64_t b = (n + 255) / 256;
    b = b < 1 ? 1 : (b > 4096 ? 4096 : b);
    hipLaunchKernelGGL(k_cache_init, dim3((unsigned)b), dim3(256), 0, s, c, n_keys, n_dir);
    return hipGetLastError();
}

hipError_t launch_vpt_update(const CacheDev& c, const CacheGeom& g, const uint32_t* gate, hipStream_t s) {
    hipLaunchKernelGGL(k_vpt_update, dim3(1), dim3(1024), 0, s, c, g, gate);
    return hipGetLastError();
}

hipError_t launch_clear_last_req(const CacheDev& c, int64_t n_keys, hipStream_t s) {
    int64_t b = (n_keys + 255) / 256;
    b = b < 1 ? 1 : (b > 4096 ? 4096 : b);
    hipLaunchKernelGGL(k_clear_last_req, dim3((unsigned)b), dim3(256), 0, s, c, n_keys);
    return hipGetLastError();
}

hipError_t launch_topk(const TopkArgs& base, const TopkPlan& plan, uint64_t* buf0, uint64_t* buf1, uint64_t* final_out,
                       const SelectArgs* epilogue, uint32_t* fuse_done, hipStream_t s) {
    if (fuse_done && plan.n_pass >= 2) {
        // one launch: pass 0, then the later passes in its last workgroup
        TopkArgs a = base;
        a.pass = 0;
        a.out = buf0;
        a.out2 = buf1;
        a.final_out = final_out;
        a.fused = 1;
        a.done = fuse_done;
        a.sel = epilogue ? *epilogue : SelectArgs{};
        hipLaunchKernelGGL(k_topk, dim3(plan.blocks[0]), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const uint64_t* src = base.in;
    for (int p = 0; p < plan.n_pass; ++p) {
        TopkArgs a = base;
        a.pass = p;
        a.in = src;
        const bool last = p + 1 == plan.n_pass;
        a.out = last ? final_out : ((p & 1) ? buf1 : buf0);
        a.final_out = final_out;
        a.last_pass = plan.n_pass - 1;
        a.sel = epilogue ? *epilogue : SelectArgs{};
        hipLaunchKernelGGL(k_topk, dim3(plan.blocks[p]), dim3(256), 0, s, a);
        src = a.out;
    }
    return hipGetLastError();
}

hipError_t launch_prefill_setup(const CacheDev& c, const CacheGeom& g, const int32_t* keys, int32_t n, int32_t stamp,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_prefill_setup, dim3(1), dim3(256), 0, s, c, g, keys, n, stamp);
    return hipGetLastError();
}

hipError_t launch_insert(const CacheDev& c, const CacheGeom& g, int32_t cap, const uint32_t* gate, hipStream_t s) {
    if (cap <= 256) {
        hipLaunchKernelGGL(k_insert, dim3(1), dim3(256), 0, s, c, g, 1, gate);
        return hipGetLastError();
    }
    int b = (cap + 255) / 256;
    b = b > 1024 ? 1024 : b;
    hipLaunchKernelGGL(k_insert, dim3(b), dim3(256), 0, s, c, g, 0, gate);
    hipLaunchKernelGGL(k_insert_finish, dim3(1), dim3(64), 0, s, c, gate);
    return hipGetLastError();
}

}  // namespace cinr
