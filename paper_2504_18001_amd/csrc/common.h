// Internal definitions shared by the HIP sources of libcinr (gfx950 only).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cinr.h"

namespace cinr {

constexpr int kMaxLevels = CINR_MAX_LEVELS;
constexpr int kMaxLods = CINR_MAX_LODS;
constexpr int kBlock = 256;  // threads per workgroup (4 wave64s)

constexpr uint32_t kPrime1 = 2654435761u;
constexpr uint32_t kPrime2 = 805459861u;

// One hash-grid level as seen by the kernels.
struct LevelDev {
    double res;       // N_l
    uint32_t side;    // N_l + 1
    uint32_t side2;   // (N_l + 1)^2
    uint32_t offset;  // first table entry of the level
    uint32_t mask;    // T - 1 for a hashed level, 0 for a dense one
};

// Hash-grid INR as seen by the kernels (passed by value).
struct InrDev {
    int32_t dims[3];
    float vm1[3];          // V - 1
    double inv_dims[3];    // 1 / V
    int32_t n_levels, n_features;
    LevelDev lv[kMaxLevels];
    float value_scale, value_offset;
    const float* table;
    const float* weights;
    int32_t in, hidden;            // widths[0], hidden width
    const float* grid;             // explicit-grid source (f32 [Vz][Vy][Vx]); null for an INR
};

// Exact unsigned division by a frame-invariant divisor d >= 1 for dividends
// n < 2^31: q = umulhi(n, ceil(2^(32+s)/d)) >> s with 2^s <= d < 2^(s+1)
// (the rounding error of the multiplier stays below one quotient step for
// n < 2^31); powers of two use a shift (mul = 0).
struct FastDiv {
    uint32_t mul;
    uint32_t shift;
};

inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t s = 0;
    while ((2u << s) <= d && s < 31) ++s;  // 2^s <= d < 2^(s+1)
    if ((d & (d - 1)) == 0) return FastDiv{0u, s};
    const unsigned __int128 num = (unsigned __int128)1 << (32 + s);
    const uint64_t m = (uint64_t)((num + d - 1) / d);
    return FastDiv{(uint32_t)m, s};
}

__device__ inline uint32_t fast_div(uint32_t n, FastDiv f) {
    return f.mul ? (__umulhi(n, f.mul) >> f.shift) : (n >> f.shift);
}

// Two-level page table (the virtualised page tables of Section 4.3.1): a
// directory entry per block of 8^3 bricks of a LoD, pointing to a block of
// 512 slot entries held in a block pool (or -1 when none of the block's
// bricks is mapped).
constexpr int kVptShift = 3;                // block side 2^3 bricks
constexpr int kVptEntries = 1 << (3 * kVptShift);

// LoD lattice / brick geometry (Section 4.3.2).
struct LodGeom {
    int32_t K[3];    // lattice points per axis
    int32_t nb[3];   // bricks per axis
    int64_t off;     // first key of the LoD
    int32_t dnb[2];  // page-table blocks along x and y
    int64_t doff;    // first directory entry of the LoD (within a volume)
};

// Keys of a cache shared by n_vols volumes of the same dimensions: volume v
// owns keys [v * keys_per_vol, (v + 1) * keys_per_vol), numbered LoD by LoD.
// Where decoded bricks go: brick r to slot slots[r] (or r), slots below
// `split` as binary32 at out + slot * B^3, the others as binary16 (rounded
// to nearest even) at out16 + (slot - split) * B^3.
struct BrickOut {
    void* out;
    void* out16;
    int32_t split;
};

// Launch shape of brick decoding: parts per brick and the LDS budget (floats)
// of the staged corner boxes; parts = 0 decodes without staging.
struct DecodeShape {
    int32_t parts = 0;
    int32_t stage_floats = 0;
};

struct CacheGeom {
    int32_t brick;
    FastDiv div_b1;  // division by brick - 1
    int32_t n_lods;
    LodGeom lod[kMaxLods];
    int64_t keys_per_vol;
    int32_t n_vols;
    int64_t n_keys;  // n_vols * keys_per_vol
    int64_t dir_per_vol;  // directory entries of the two-level page table per volume
};

// Directory entry and block entry of brick b (coordinates at LoD lg) within
// its volume's directory.
__host__ __device__ inline int64_t vpt_dir(const LodGeom& lg, const int32_t b[3]) {
    return lg.doff + ((int64_t)(b[2] >> kVptShift) * lg.dnb[1] + (b[1] >> kVptShift)) * lg.dnb[0] + (b[0] >> kVptShift);
}
__host__ __device__ inline int32_t vpt_entry(const int32_t b[3]) {
    constexpr int32_t m = (1 << kVptShift) - 1;
    return (((b[2] & m) << kVptShift | (b[1] & m)) << kVptShift) | (b[0] & m);
}

// Directory entry (over all volumes) and block entry of a brick key.
__host__ __device__ inline void vpt_addr(const CacheGeom& g, int64_t key, int64_t* d, int32_t* e) {
    const int64_t vol = key / g.keys_per_vol;
    const int64_t vkey = key - vol * g.keys_per_vol;
    int32_t L = 0;
    while (L + 1 < g.n_lods && vkey >= g.lod[L + 1].off) ++L;
    const LodGeom& lg = g.lod[L];
    const int64_t local = vkey - lg.off;
    int32_t b[3];
    b[0] = (int32_t)(local % lg.nb[0]);
    b[1] = (int32_t)((local / lg.nb[0]) % lg.nb[1]);
    b[2] = (int32_t)(local / ((int64_t)lg.nb[0] * lg.nb[1]));
    *d = vol * g.dir_per_vol + vpt_dir(lg, b);
    *e = vpt_entry(b);
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------

__device__ inline int lane_id() { return __lane_id(); }

// Wave-aggregated append: returns the index of this lane's element in the
// destination list, or -1 when `pred` is false.  One atomic per wave.
__device__ inline int64_t wave_append(bool pred, uint32_t* counter) {
    const uint64_t mask = __ballot(pred);
    if (!pred) return -1;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    const uint32_t rank = __popcll(mask & ((1ull << lane_id()) - 1ull));
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    return (int64_t)base + rank;
}

// Reserves n consecutive entries per lane of a list with one atomic per wave
// and returns this lane's first index.  All 64 lanes must call it together
// (lanes with nothing to add pass n = 0).
__device__ inline uint32_t wave_reserve(uint32_t n, uint32_t* counter) {
    uint32_t incl = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o);
        if (lane_id() >= o) incl += v;
    }
    const uint32_t total = __shfl(incl, 63);
    uint32_t base = 0;
    if (lane_id() == 63 && total) base = atomicAdd(counter, total);
    base = __shfl(base, 63);
    return base + incl - n;
}

// Wave-aggregated 64-bit counter increment.
__device__ inline void wave_add_u64(unsigned long long* dst, uint64_t v) {
    // reduce across the wave with shuffles
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

inline hipError_t launch_check() { return hipGetLastError(); }

// Philox-4x32-10 (Salmon et al. 2011): counter c (in place), key (k0, k1).
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

}  // namespace cinr
