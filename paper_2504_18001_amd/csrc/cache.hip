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
#include "frame.h"

namespace cinr {

__global__ void k_cache_init(CacheDev c, int64_t n_keys) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_keys; t += stride) {
        c.pt[t] = -1;
        c.rank[t] = -1;
        c.req[t] = 0u;
        if (c.last_req) c.last_req[t] = 0u;
    }
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < c.pool_bricks; t += stride) {
        c.owner[t] = -1;
        c.last_used[t] = -1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *c.ctr = CacheCtr{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
}

__global__ void k_cm_rank(CacheDev c, int32_t frame) {
    const uint32_t n = c.ctr->n_touched;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t key = c.touched[i];
        const uint32_t cnt = c.req[key];
        if (c.last_req) c.last_req[key] = cnt;
        const int64_t old = c.rank[key];
        int64_t r = old < 0 ? (int64_t)frame + (int64_t)cnt - 1 : old + (int64_t)cnt;
        const int64_t cap = (int64_t)frame + c.rank_window;
        if (r > cap) r = cap;
        c.rank[key] = r;
        c.req[key] = 0u;
        const uint64_t low = 0xFFFFFFFFull - (uint64_t)(uint32_t)key;
        c.cand[i] = c.ranking ? (((uint64_t)r << 32) | low) : low;
    }
}

// Clears the request counts kept for dumps (before the frame's sampler).
__global__ void k_clear_last_req(CacheDev c, int64_t n_keys) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_keys; t += (int64_t)gridDim.x * blockDim.x)
        c.last_req[t] = 0u;
}

// One tournament pass: workgroup b sorts elements [b*2048, (b+1)*2048) of
// its input (missing elements are 0, which sorts last) in descending order
// and writes the first k to out[b*k ...].  In LRU mode the input is the slot
// range [0, count) scored ~(last_used << 32 | slot).
__global__ __launch_bounds__(256) void k_topk(const uint64_t* in, const uint32_t* count_dev, uint32_t count_cap,
                                              uint64_t* out, int32_t k, const uint32_t* gate,
                                              const int32_t* lru_last_used) {
    __shared__ uint64_t s[kTopkChunk];
    if (gate && *gate == 0u) return;
    uint32_t count = count_cap;
    if (count_dev && *count_dev < count) count = *count_dev;
    const uint64_t base = (uint64_t)blockIdx.x * kTopkChunk;
    for (int e = threadIdx.x; e < kTopkChunk; e += 256) {
        const uint64_t idx = base + e;
        uint64_t v = 0ull;
        if (idx < count) {
            if (lru_last_used)
                v = ~(((uint64_t)(uint32_t)lru_last_used[idx] << 32) | (uint64_t)idx);
            else
                v = in[idx];
        }
        s[e] = v;
    }
    __syncthreads();
    for (int len = 2; len <= kTopkChunk; len <<= 1) {
        for (int j = len >> 1; j > 0; j >>= 1) {
            for (int e = threadIdx.x; e < kTopkChunk; e += 256) {
                const int x = e ^ j;
                if (x > e) {
                    const uint64_t a = s[e], b = s[x];
                    const bool desc = (e & len) == 0;
                    if (desc ? (a < b) : (a > b)) {
                        s[e] = b;
                        s[x] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < k; e += 256) out[(uint64_t)blockIdx.x * k + e] = s[e];
}

// Request list from the final selection; free-slot and eviction counts.
__global__ void k_cm_select(CacheDev c) {
    const int32_t lim = c.max_requests < c.pool_bricks ? c.max_requests : c.pool_bricks;
    __shared__ uint32_t nsel;
    if (threadIdx.x == 0) nsel = 0u;
    __syncthreads();
    for (int32_t t = threadIdx.x; t < lim; t += blockDim.x) {
        const uint64_t v = c.sel[t];
        if (v != 0ull) {
            c.ins_keys[t] = (int32_t)(0xFFFFFFFFull - (v & 0xFFFFFFFFull));
            atomicAdd(&nsel, 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        CacheCtr* ctr = c.ctr;
        const uint32_t n_free = (uint32_t)c.pool_bricks - ctr->n_used;
        ctr->n_sel = nsel;
        ctr->n_free = n_free;
        ctr->need_evict = nsel > n_free ? nsel - n_free : 0u;
    }
}

// Prefill: the given keys are inserted into free slots only.
__global__ void k_prefill_setup(CacheDev c, const int32_t* keys, int32_t n) {
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) c.ins_keys[t] = keys[t];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        CacheCtr* ctr = c.ctr;
        const uint32_t n_free = (uint32_t)c.pool_bricks - ctr->n_used;
        const uint32_t nn = (uint32_t)n <= n_free ? (uint32_t)n : n_free;
        if ((uint32_t)n > n_free) ctr->error |= 1u;
        ctr->n_sel = nn;
        ctr->n_free = n_free;
        ctr->need_evict = 0u;
    }
}

__global__ void k_insert(CacheDev c, CacheGeom g, int32_t stamp) {
    const CacheCtr ctr = *c.ctr;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ctr.n_sel; t += gridDim.x * blockDim.x) {
        const int32_t key = c.ins_keys[t];
        int32_t slot;
        if (t < ctr.n_free)
            slot = (int32_t)(ctr.n_used + t);
        else
            slot = (int32_t)(uint32_t)(~c.vic[t - ctr.n_free] & 0xFFFFFFFFull);
        bool ok = key >= 0 && (int64_t)key < g.n_keys && slot >= 0 && slot < c.pool_bricks;
        int32_t old = -1;
        if (ok) {
            old = c.owner[slot];
            if (old >= 0) {
                c.pt[old] = -1;
                c.rank[old] = -1;
            }
            c.pt[key] = slot;
            c.owner[slot] = key;
            c.last_used[slot] = stamp;
        }
        // brick coordinates of the key
        int32_t L = 0;
        while (L + 1 < g.n_lods && (int64_t)key >= g.lod[L + 1].off) ++L;
        const int64_t local = ok ? (int64_t)key - g.lod[L].off : 0;
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

__global__ void k_insert_finish(CacheDev c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        CacheCtr* ctr = c.ctr;
        const uint32_t filled = ctr->n_sel < ctr->n_free ? ctr->n_sel : ctr->n_free;
        ctr->n_used += filled;
        ctr->n_evlog += ctr->n_sel;
    }
}

__global__ void k_touched_reset(CacheDev c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c.ctr->n_touched = 0u;
}

// ---------------------------------------------------------------------------

hipError_t launch_cache_init(const CacheDev& c, int64_t n_keys, hipStream_t s) {
    int64_t n = n_keys > c.pool_bricks ? n_keys : c.pool_bricks;
    int64_t b = (n + 255) / 256;
    b = b < 1 ? 1 : (b > 4096 ? 4096 : b);
    hipLaunchKernelGGL(k_cache_init, dim3((unsigned)b), dim3(256), 0, s, c, n_keys);
    return hipGetLastError();
}

hipError_t launch_clear_last_req(const CacheDev& c, int64_t n_keys, hipStream_t s) {
    int64_t b = (n_keys + 255) / 256;
    b = b < 1 ? 1 : (b > 4096 ? 4096 : b);
    hipLaunchKernelGGL(k_clear_last_req, dim3((unsigned)b), dim3(256), 0, s, c, n_keys);
    return hipGetLastError();
}

hipError_t launch_cm_rank(const CacheDev& c, int32_t frame, int64_t cap, hipStream_t s) {
    int64_t b = (cap + 255) / 256;
    b = b < 1 ? 1 : (b > 1024 ? 1024 : b);
    hipLaunchKernelGGL(k_cm_rank, dim3((unsigned)b), dim3(256), 0, s, c, frame);
    return hipGetLastError();
}

hipError_t launch_topk(const uint64_t* in, const uint32_t* count_dev, const TopkPlan& plan, int k, uint64_t* buf0,
                       uint64_t* buf1, uint64_t* final_out, const uint32_t* gate, const int32_t* lru_last_used,
                       hipStream_t s) {
    const uint64_t* src = in;
    for (int p = 0; p < plan.n_pass; ++p) {
        uint64_t* dst = (p + 1 == plan.n_pass) ? final_out : ((p & 1) ? buf1 : buf0);
        hipLaunchKernelGGL(k_topk, dim3(plan.blocks[p]), dim3(256), 0, s, src, p == 0 ? count_dev : nullptr,
                           plan.count[p], dst, k, gate, p == 0 ? lru_last_used : nullptr);
        src = dst;
    }
    return hipGetLastError();
}

hipError_t launch_cm_select(const CacheDev& c, hipStream_t s) {
    hipLaunchKernelGGL(k_cm_select, dim3(1), dim3(1024), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_prefill_setup(const CacheDev& c, const int32_t* keys, int32_t n, hipStream_t s) {
    int b = (n + 255) / 256;
    b = b < 1 ? 1 : (b > 1024 ? 1024 : b);
    hipLaunchKernelGGL(k_prefill_setup, dim3(b), dim3(256), 0, s, c, keys, n);
    return hipGetLastError();
}

hipError_t launch_insert(const CacheDev& c, const CacheGeom& g, int32_t stamp, int32_t cap, hipStream_t s) {
    int b = (cap + 255) / 256;
    b = b < 1 ? 1 : (b > 1024 ? 1024 : b);
    hipLaunchKernelGGL(k_insert, dim3(b), dim3(256), 0, s, c, g, stamp);
    hipLaunchKernelGGL(k_insert_finish, dim3(1), dim3(64), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_touched_reset(const CacheDev& c, hipStream_t s) {
    hipLaunchKernelGGL(k_touched_reset, dim3(1), dim3(64), 0, s, c);
    return hipGetLastError();
}

}  // namespace cinr
