// Hash-grid INR evaluation on gfx950: encoding on the vector ALUs, the MLP on
// MFMA (Section 3, Figure 2).  Used by brick decoding (Section 4.3.2), true-
// miss inference (Section 4.3.4, Algorithm 1) and the uncached renderer.
//
// Layout of one round (a workgroup of 256 lanes = 4 wave64s, 256 points):
//  - each lane encodes one point over all levels (level constants are
//    wave-uniform, so dense/hashed branches never diverge) and writes its
//    feature row to LDS;
//  - each wave then runs its 64 points through the MLP as four 16-point MFMA
//    tiles.  Layers are computed transposed (H^T = W X^T): weights are the
//    A operand (rows = neurons), points the B operand (columns), so a layer's
//    accumulator (lane l: neurons 4*(l/16)+r of point l%16) is directly the
//    next layer's B operand once the K order of the next weight matrix is
//    permuted to match.  Hidden activations never leave registers.
//  - the last layer (width 1) is a per-lane dot product in FP32 reduced across
//    the four 16-lane groups; lane l ends with the output of point l.
#include <type_traits>

#include "common.h"
#include "inr_engine.h"

namespace cinr {

// ---------------------------------------------------------------------------
// Point sources and sinks
// ---------------------------------------------------------------------------

// Arbitrary positions (voxel coordinates, f32 xyz).
struct PosSrc {
    const float* pos;
    int64_t n;
    __device__ int64_t count() const { return n; }
    __device__ void position(int64_t i, double x[3]) const {
        x[0] = pos[3 * i];
        x[1] = pos[3 * i + 1];
        x[2] = pos[3 * i + 2];
    }
};

struct LinearDst {
    float* out;
    __device__ void store(int64_t i, float v) const { out[i] = v; }
};

// Brick lattice points: request r = (lod, bx, by, bz), sample i in (z, y, x)
// order; voxel coordinate clamp((b*(B-1) + i) * 2^lod, 0, V-1).
struct BrickSrc {
    const int32_t* reqs;      // [n][4]
    const uint32_t* n_dev;    // device count of requests (nullable)
    const uint32_t* gate;     // nullable: no request unless *gate != 0
    int32_t n_host;
    int32_t B;
    int32_t B3;
    int32_t n_lods;
    int32_t nb[kMaxLods][3];
    int32_t dims[3];
    __device__ int64_t n_requests() const {
        if (gate && *gate == 0u) return 0;
        return n_dev ? (int64_t)*n_dev : (int64_t)n_host;
    }
    __device__ int64_t count() const { return n_requests() * B3; }
    // Voxel coordinate along axis a of lattice index i of request r (the
    // per-axis part of position); *ok as position's result.
    __device__ double axis_x(int64_t r, int a, int32_t i, bool* ok) const {
        const int32_t* q = reqs + 4 * r;
        const int32_t L = q[0];
        const bool okl = L >= 0 && L < n_lods;
        const int32_t Ls = okl ? L : 0;
        const int32_t b = q[1 + a];
        const bool ba = b >= 0 && b < nb[Ls][a];
        int64_t xa = ((int64_t)(ba ? b : 0) * (B - 1) + i) << Ls;
        if (xa > dims[a] - 1) xa = dims[a] - 1;
        *ok = okl && ba;
        return (double)xa;
    }
    // returns false for an invalid request
    __device__ bool position(int64_t idx, double x[3]) const {
        const int32_t r = (int32_t)(idx / B3);
        const int32_t i = (int32_t)(idx - (int64_t)r * B3);
        const int32_t* q = reqs + 4 * r;
        const int32_t L = q[0];
        const int32_t ix = i % B, iy = (i / B) % B, iz = i / (B * B);
        const int32_t li[3] = {ix, iy, iz};
        bool ok = L >= 0 && L < n_lods;
        const int32_t Ls = ok ? L : 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int32_t b = q[1 + a];
            const bool ba = b >= 0 && b < nb[Ls][a];
            ok = ok && ba;
            int64_t xa = ((int64_t)(ba ? b : 0) * (B - 1) + li[a]) << Ls;
            if (xa > dims[a] - 1) xa = dims[a] - 1;
            x[a] = (double)xa;
        }
        return ok;
    }
};

struct BrickDst {
    void* out;             // binary32 slots [0, split)
    void* out16;           // binary16 slots [split, ...), rounded to nearest even
    const int32_t* slots;  // nullable: brick r goes to slot slots[r] (skipped if negative), else to r
    int32_t B3;
    int32_t split;
    __device__ void store(int64_t idx, float v) const {
        const int32_t r = (int32_t)(idx / B3);
        const int32_t i = (int32_t)(idx - (int64_t)r * B3);
        const int64_t s = slots ? (int64_t)slots[r] : (int64_t)r;
        if (s < 0) return;
        if (s >= split)
            static_cast<__half*>(out16)[(s - split) * B3 + i] = __float2half_rn(v);
        else
            static_cast<float*>(out)[s * B3 + i] = v;
    }
};

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

template <class Eng, class Src, class Dst>
__global__ __launch_bounds__(kBlock) void k_inr_points(const InrDev m, const Src src, const Dst dst) {
    const int64_t n = src.count();
    // grids are sized for a capacity: a workgroup with no point leaves before
    // loading the weights (the count is the same for the whole workgroup)
    if ((int64_t)blockIdx.x * kBlock >= n) return;
    Eng eng;
    eng.load_weights(m);
    __shared__ typename Eng::Lds lds;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
        const int64_t idx = base + threadIdx.x;
        const bool valid = idx < n;
        double x[3];
        src.position(valid ? idx : base, x);
        const float v = eng.eval(m, x, lds);
        if (valid) dst.store(idx, v);
    }
}

// Brick decoding: like k_inr_points, invalid requests produce NaN bricks.
template <class Eng>
__global__ __launch_bounds__(kBlock) void k_decode(const InrDev m, const BrickSrc src, const BrickDst dst) {
    const int64_t n = src.count();
    // launched for the frame's request cap: with fewer (or no) selected
    // bricks, idle workgroups leave before loading the weights
    if ((int64_t)blockIdx.x * kBlock >= n) return;
    Eng eng;
    eng.load_weights(m);
    __shared__ typename Eng::Lds lds;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
        const int64_t idx = base + threadIdx.x;
        const bool valid = idx < n;
        double x[3];
        const bool ok = src.position(valid ? idx : base, x);
        const float v = eng.eval(m, x, lds);
        if (valid) dst.store(idx, ok ? v : __builtin_nanf(""));
    }
}

// Persistent decoding of the bricks of several volumes of one shape (a cache
// shared by several INRs): workgroup rounds walk (brick, 256-sample chunk)
// items, so that every round stays inside one brick; a workgroup reloads the
// MLP weights only when its next brick belongs to another volume.  The list
// may mix volumes and LoDs in any order.
// Brick decoding by parts of bricks.  Work item = one part of a brick
// (`parts` parts of B/parts z-slices each, B <= 16), all 256 lanes.  The
// lattice coordinates of a brick are separable, so each level's cells and
// weights along each axis are computed once per item (the same FP64
// operations as for a single point) into a table in LDS.  With
// kStageFloats > 0, the grid corners the part's lattice points touch form a
// box per level (from the part's first and last points: the lattice
// coordinates, u and the cell index are all monotone); boxes are staged in
// LDS smallest first while they fit in kStageFloats floats and cost fewer
// reads than the points' own corner reads.  Every variant gives the same bits
// (same cells, weights and order).  vol_ok false gives NaN (a request of no
// volume).
constexpr int kTabB = 16;  // largest brick side of the per-axis tables
template <class Eng, int kStageFloats>
__device__ void decode_item_staged(const InrDev& m, Eng& eng, typename Eng::Lds& lds, float* stage, StageLevel* sl,
                                   int64_t* vol_s, uint2* ctab, const BrickSrc& src, const BrickDst& dst, int64_t r,
                                   int32_t part, int32_t parts, bool vol_ok) {
    constexpr int F = Eng::F;
    const int NL = m.n_levels;
    const int32_t B = src.B, per = src.B3 / parts, first = part * per;
    const int64_t i0 = r * src.B3 + first;
    for (int t = threadIdx.x; t < NL * 3 * B; t += kBlock) {
        const int l = t / (3 * B), rem = t - l * 3 * B, a = rem / B, i = rem - a * B;
        bool ok;
        double xa = src.axis_x(r, a, i, &ok);
        xa = xa < 0.0 ? 0.0 : xa;
        xa = xa > (double)m.vm1[a] ? (double)m.vm1[a] : xa;
        const double u = (xa + 0.5) * m.inv_dims[a];
        const double sa = u * m.lv[l].res;
        const double fa = floor(sa);
        ctab[t] = make_uint2((uint32_t)fa, __float_as_uint((float)(sa - fa)));
    }
    if (kStageFloats > 0 && (int)threadIdx.x < NL) {
        double xa[3], xb[3], ua[3], ub[3];
        src.position(i0, xa);
        src.position(i0 + per - 1, xb);
        to_unit(m, xa, ua);
        to_unit(m, xb, ub);
        const LevelDev& lv = m.lv[threadIdx.x];
        StageLevel q;
        int64_t vol = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q.lo[a] = (int32_t)floor(ua[a] * lv.res);
            q.e[a] = (int32_t)floor(ub[a] * lv.res) + 2 - q.lo[a];
            vol *= q.e[a];
        }
        q.off = -1;
        sl[threadIdx.x] = q;
        vol_s[threadIdx.x] = vol;
    }
    __syncthreads();
    if (kStageFloats > 0) {
        if (threadIdx.x == 0) {
            uint32_t taken = 0u;
            int64_t used = 0;
            for (int k = 0; k < NL; ++k) {
                int best = -1;
                for (int l = 0; l < NL; ++l)
                    if (!((taken >> l) & 1u) && (best < 0 || vol_s[l] < vol_s[best])) best = l;
                taken |= 1u << best;
                const int64_t need = (vol_s[best] * F + 3) & ~(int64_t)3;
                if (used + need <= kStageFloats && vol_s[best] < 8 * (int64_t)per) {
                    sl[best].off = (int32_t)used;
                    used += need;
                }
            }
        }
        __syncthreads();
        for (int l = 0; l < NL; ++l) {
            const StageLevel q = sl[l];
            if (q.off < 0) continue;
            const LevelDev& lv = m.lv[l];
            const int32_t ex = q.e[0], exy = q.e[0] * q.e[1], vol = exy * q.e[2];
            const float* tb = m.table + (size_t)lv.offset * F;
            for (int32_t k = threadIdx.x; k < vol; k += kBlock) {
                const int32_t cz = k / exy, rem = k - cz * exy, cy = rem / ex, cx = rem - cy * ex;
                const uint32_t c0 = (uint32_t)(q.lo[0] + cx), c1 = (uint32_t)(q.lo[1] + cy),
                               c2 = (uint32_t)(q.lo[2] + cz);
                const uint32_t idx = lv.mask == 0u ? c0 + c1 * lv.side + c2 * lv.side2
                                                   : (c0 ^ (c1 * kPrime1) ^ (c2 * kPrime2)) & lv.mask;
                float e[F];
                Entry<F>::load(tb + (size_t)idx * F, e);
#pragma unroll
                for (int j = 0; j < F; ++j) stage[q.off + k * F + j] = e[j];
            }
        }
        __syncthreads();
    }
    double x0[3];
    const bool ok = src.position(i0, x0) && vol_ok;  // the request's validity (the same for all its points)
    for (int32_t b0 = 0; b0 < per; b0 += kBlock) {
        const int32_t i = b0 + (int32_t)threadIdx.x;
        const bool valid = i < per;
        const int32_t gi = first + (valid ? i : 0);
        CoordTab co;
        co.tab = ctab;
        co.n = B;
        co.i[0] = gi % B;
        co.i[1] = (gi / B) % B;
        co.i[2] = gi / (B * B);
        const float v = eng.eval_c(m, co, lds, kStageFloats > 0 ? sl : nullptr, stage);
        if (valid) dst.store(i0 + i, ok ? v : __builtin_nanf(""));
    }
    __syncthreads();  // the tables, stage and boxes are refilled for the next item
}

// Parts per brick of a launch: at least `parts`; doubled (while it divides the
// brick) until the request count read on the device gives every workgroup of
// the grid an item, so that a short request list still fills the chip.
__device__ inline int32_t decode_parts(int64_t n, int32_t parts, int32_t B) {
    int32_t p = parts;
    while (2 * p <= kTabB && B % (2 * p) == 0 && n * p < (int64_t)gridDim.x) p *= 2;
    return p;
}

template <class Eng, int kStageFloats>
__global__ __launch_bounds__(kBlock) void k_decode_staged(const InrDev m, const BrickSrc src, const BrickDst dst,
                                                          int32_t min_parts) {
    const int64_t n = src.n_requests();
    const int32_t parts = decode_parts(n, min_parts, src.B);
    const int64_t items = n * parts;
    // sized for the request cap: idle workgroups leave before the weights
    if ((int64_t)blockIdx.x >= items) return;
    Eng eng;
    eng.load_weights(m);
    __shared__ typename Eng::Lds lds;
    __shared__ float stage[kStageFloats > 0 ? kStageFloats : 1];
    __shared__ StageLevel sl[kMaxLevels];
    __shared__ int64_t vol_s[kMaxLevels];
    __shared__ uint2 ctab[kMaxLevels * 3 * kTabB];
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t r = it / parts;
        decode_item_staged<Eng, kStageFloats>(m, eng, lds, stage, sl, vol_s, ctab, src, dst, r,
                                              (int32_t)(it - r * parts), parts, true);
    }
}

// The same over the bricks of several volumes of one shape (a shared cache):
// request r belongs to volume req_vol[r]; weights are reloaded when a
// workgroup's volume changes.
template <class Eng, int kStageFloats>
__global__ __launch_bounds__(kBlock) void k_decode_staged_multi(const InrDev* vols, const BrickSrc src,
                                                                const int32_t* req_vol, const BrickDst dst,
                                                                int32_t min_parts) {
    const int64_t n = src.n_requests();
    const int32_t parts = decode_parts(n, min_parts, src.B);
    const int64_t items = n * parts;
    if ((int64_t)blockIdx.x >= items) return;
    Eng eng;
    int32_t cur = -1;
    __shared__ typename Eng::Lds lds;
    __shared__ float stage[kStageFloats > 0 ? kStageFloats : 1];
    __shared__ StageLevel sl[kMaxLevels];
    __shared__ int64_t vol_s[kMaxLevels];
    __shared__ uint2 ctab[kMaxLevels * 3 * kTabB];
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t r = it / parts;
        const int32_t v = req_vol[r];
        const InrDev& m = vols[v < 0 ? 0 : v];
        if (v != cur) {
            eng.load_weights(m);
            cur = v;
        }
        decode_item_staged<Eng, kStageFloats>(m, eng, lds, stage, sl, vol_s, ctab, src, dst, r,
                                              (int32_t)(it - r * parts), parts, v >= 0);
    }
}

template <class Eng>
__global__ __launch_bounds__(kBlock) void k_decode_multi(const InrDev* vols, const BrickSrc src, const int32_t* req_vol,
                                                         const BrickDst dst) {
    Eng eng;
    int32_t cur = -1;
    __shared__ typename Eng::Lds lds;
    const int64_t n_bricks = src.n_requests();
    const int32_t chunks = (src.B3 + kBlock - 1) / kBlock;
    const int64_t items = n_bricks * chunks;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t r = it / chunks;
        const int32_t i = (int32_t)(it - r * chunks) * kBlock + threadIdx.x;
        const bool valid = i < src.B3;
        const int64_t idx = r * src.B3 + (valid ? i : 0);
        const int32_t v = req_vol[r];
        const InrDev& m = vols[v < 0 ? 0 : v];
        if (v != cur) {
            eng.load_weights(m);
            cur = v;
        }
        double x[3];
        const bool ok = src.position(idx, x) && v >= 0;
        const float val = eng.eval(m, x, lds);
        if (valid) dst.store(idx, ok ? val : __builtin_nanf(""));
    }
}

// Macro-cells (Section 5.2): one workgroup per cell, min/max of the lattice
// values in the cell's closed region.
template <class Eng>
__global__ __launch_bounds__(kBlock) void k_macrocells(const InrDev m, int32_t N, int32_t Mx, int32_t My,
                                                       int32_t Mz, float* minmax) {
    Eng eng;
    eng.load_weights(m);
    __shared__ typename Eng::Lds lds;
    __shared__ float red[2][kBlock / 64];
    const int64_t ncell = (int64_t)Mx * My * Mz;
    for (int64_t c = blockIdx.x; c < ncell; c += gridDim.x) {
        const int32_t cx = (int32_t)(c % Mx), cy = (int32_t)((c / Mx) % My), cz = (int32_t)(c / ((int64_t)Mx * My));
        const int32_t lo[3] = {cx * N, cy * N, cz * N};
        int32_t ext[3];
        const int32_t ci[3] = {cx, cy, cz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int32_t hi = (ci[a] + 1) * N;
            if (hi > m.dims[a] - 1) hi = m.dims[a] - 1;
            ext[a] = hi - lo[a] + 1;
        }
        const int32_t npts = ext[0] * ext[1] * ext[2];
        float vmin = __builtin_inff(), vmax = -__builtin_inff();
        for (int32_t base = 0; base < npts; base += kBlock) {
            const int32_t i = base + threadIdx.x;
            const bool valid = i < npts;
            const int32_t j = valid ? i : base;
            double x[3] = {(double)(lo[0] + j % ext[0]), (double)(lo[1] + (j / ext[0]) % ext[1]),
                           (double)(lo[2] + j / (ext[0] * ext[1]))};
            const float v = eng.eval(m, x, lds);
            if (valid) {
                vmin = fminf(vmin, v);
                vmax = fmaxf(vmax, v);
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            vmin = fminf(vmin, __shfl_xor(vmin, o));
            vmax = fmaxf(vmax, __shfl_xor(vmax, o));
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = vmin;
            red[1][threadIdx.x >> 6] = vmax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float a = red[0][0], b = red[1][0];
            for (int w = 1; w < kBlock / 64; ++w) {
                a = fminf(a, red[0][w]);
                b = fmaxf(b, red[1][w]);
            }
            minmax[2 * c] = a;
            minmax[2 * c + 1] = b;
        }
        __syncthreads();
    }
}

// True misses of the cached renderer: records (x, y, z, destination index).
struct MissSrc {
    const float4* rec;
    const uint32_t* n_dev;
    __device__ int64_t count() const { return (int64_t)*n_dev; }
    __device__ void position(int64_t i, double x[3]) const {
        const float4 r = rec[i];
        x[0] = r.x;
        x[1] = r.y;
        x[2] = r.z;
    }
};

struct MissDst {
    const float4* rec;
    float* vals;
    __device__ void store(int64_t i, float v) const { vals[__float_as_uint(rec[i].w)] = v; }
};

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------

static int grid_for(int64_t points, int max_blocks) {
    int64_t b = (points + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

constexpr int kMaxInrBlocks = 256 * 8;  // 8 workgroups per CU on 256 CUs

// Workgroups of `kernel` resident on the current device at once (per
// instantiation and device), at least 1.
template <class Kernel>
static int resident_grid(Kernel kernel, int* cache) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return kMaxInrBlocks;
    if (cache[dev] == 0) {
        int per_cu = 0, n_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return kMaxInrBlocks;
        cache[dev] = (per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1);
    }
    return cache[dev];
}

// Grid of a staged decoding launch: one resident wave of workgroups, or fewer
// when even `parts_max` parts of every request of the cap are fewer items.
template <class Kernel>
static int staged_grid(Kernel kernel, int* cache, int64_t n_cap, int32_t parts, int32_t B) {
    int32_t pmax = parts;
    while (2 * pmax <= kTabB && B % (2 * pmax) == 0) pmax *= 2;
    const int64_t items = n_cap * pmax;
    const int cap = resident_grid(kernel, cache);
    return (int)(items < cap ? (items < 1 ? 1 : items) : cap);
}

template <class Eng>
static hipError_t launch_all(int what, const InrDev& m, const void* a, hipStream_t s) {
    switch (what) {
        case 0: {
            const PosSrc* src = (const PosSrc*)((const void* const*)a)[0];
            const LinearDst* dst = (const LinearDst*)((const void* const*)a)[1];
            hipLaunchKernelGGL((k_inr_points<Eng, PosSrc, LinearDst>), dim3(grid_for(src->n, kMaxInrBlocks)),
                               dim3(kBlock), 0, s, m, *src, *dst);
            break;
        }
        case 1: {
            const BrickSrc* src = (const BrickSrc*)((const void* const*)a)[0];
            const BrickDst* dst = (const BrickDst*)((const void* const*)a)[1];
            const int64_t cap = (int64_t)src->n_host * src->B3;
            hipLaunchKernelGGL((k_decode<Eng>), dim3(grid_for(cap, kMaxInrBlocks)), dim3(kBlock), 0, s, m, *src,
                               *dst);
            break;
        }
        case 2: {
            const int32_t* p = (const int32_t*)((const void* const*)a)[0];
            float* mm = (float*)((const void* const*)a)[1];
            const int64_t nc = (int64_t)p[1] * p[2] * p[3];
            hipLaunchKernelGGL((k_macrocells<Eng>), dim3((int)(nc < kMaxInrBlocks * 4 ? nc : kMaxInrBlocks * 4)),
                               dim3(kBlock), 0, s, m, p[0], p[1], p[2], p[3], mm);
            break;
        }
        case 4: {
            const BrickSrc* src = (const BrickSrc*)((const void* const*)a)[0];
            const BrickDst* dst = (const BrickDst*)((const void* const*)a)[1];
            const InrDev* vols = (const InrDev*)((const void* const*)a)[2];
            const int32_t* req_vol = (const int32_t*)((const void* const*)a)[3];
            const int64_t items = (int64_t)src->n_host * ((src->B3 + kBlock - 1) / kBlock);
            const int blocks = (int)(items < kMaxInrBlocks ? (items < 1 ? 1 : items) : kMaxInrBlocks);
            hipLaunchKernelGGL((k_decode_multi<Eng>), dim3(blocks), dim3(kBlock), 0, s, vols, *src, req_vol, *dst);
            break;
        }
        case 5: {
            // LDS-staged decoding (INR engines only): a[2] = {parts, stage floats}
            const BrickSrc* src = (const BrickSrc*)((const void* const*)a)[0];
            const BrickDst* dst = (const BrickDst*)((const void* const*)a)[1];
            const int32_t* shape = (const int32_t*)((const void* const*)a)[2];
            if constexpr (std::is_same<Eng, GridEngine>::value) {
                hipLaunchKernelGGL((k_decode<Eng>), dim3(grid_for((int64_t)src->n_host * src->B3, kMaxInrBlocks)),
                                   dim3(kBlock), 0, s, m, *src, *dst);
            } else {
                static int cap0[64], cap1[64], cap2[64];
                const int64_t n = src->n_host;
                if (shape[1] <= 0)
                    hipLaunchKernelGGL((k_decode_staged<Eng, 0>),
                                       dim3(staged_grid(k_decode_staged<Eng, 0>, cap0, n, shape[0], src->B)),
                                       dim3(kBlock), 0, s, m, *src, *dst, shape[0]);
                else if (shape[1] <= 8192)
                    hipLaunchKernelGGL((k_decode_staged<Eng, 8192>),
                                       dim3(staged_grid(k_decode_staged<Eng, 8192>, cap1, n, shape[0], src->B)),
                                       dim3(kBlock), 0, s, m, *src, *dst, shape[0]);
                else
                    hipLaunchKernelGGL((k_decode_staged<Eng, 16384>),
                                       dim3(staged_grid(k_decode_staged<Eng, 16384>, cap2, n, shape[0], src->B)),
                                       dim3(kBlock), 0, s, m, *src, *dst, shape[0]);
            }
            break;
        }
        case 6: {
            // LDS-staged decoding over several volumes: a[4] = {parts, stage floats}
            const BrickSrc* src = (const BrickSrc*)((const void* const*)a)[0];
            const BrickDst* dst = (const BrickDst*)((const void* const*)a)[1];
            const InrDev* vols = (const InrDev*)((const void* const*)a)[2];
            const int32_t* req_vol = (const int32_t*)((const void* const*)a)[3];
            const int32_t* shape = (const int32_t*)((const void* const*)a)[4];
            if constexpr (std::is_same<Eng, GridEngine>::value) {
                return hipErrorInvalidValue;
            } else {
                static int cap0[64], cap1[64], cap2[64];
                const int64_t n = src->n_host;
                if (shape[1] <= 0)
                    hipLaunchKernelGGL((k_decode_staged_multi<Eng, 0>),
                                       dim3(staged_grid(k_decode_staged_multi<Eng, 0>, cap0, n, shape[0], src->B)),
                                       dim3(kBlock), 0, s, vols, *src, req_vol, *dst, shape[0]);
                else if (shape[1] <= 8192)
                    hipLaunchKernelGGL((k_decode_staged_multi<Eng, 8192>),
                                       dim3(staged_grid(k_decode_staged_multi<Eng, 8192>, cap1, n, shape[0], src->B)),
                                       dim3(kBlock), 0, s, vols, *src, req_vol, *dst, shape[0]);
                else
                    hipLaunchKernelGGL((k_decode_staged_multi<Eng, 16384>),
                                       dim3(staged_grid(k_decode_staged_multi<Eng, 16384>, cap2, n, shape[0], src->B)),
                                       dim3(kBlock), 0, s, vols, *src, req_vol, *dst, shape[0]);
            }
            break;
        }
        case 3: {
            const MissSrc* src = (const MissSrc*)((const void* const*)a)[0];
            const MissDst* dst = (const MissDst*)((const void* const*)a)[1];
            const int64_t cap = *(const int64_t*)((const void* const*)a)[2];
            hipLaunchKernelGGL((k_inr_points<Eng, MissSrc, MissDst>), dim3(grid_for(cap, kMaxInrBlocks)),
                               dim3(kBlock), 0, s, m, *src, *dst);
            break;
        }
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NL, int F, int H>
static hipError_t dispatch_prec(int prec, int what, const InrDev& m, const void* a, hipStream_t s) {
    switch (prec) {
        case CINR_F32: return launch_all<InrEngine<EngCfg<NL, F, H, CINR_F32>>>(what, m, a, s);
        case CINR_BF16: return launch_all<InrEngine<EngCfg<NL, F, H, CINR_BF16>>>(what, m, a, s);
        case CINR_F16: return launch_all<InrEngine<EngCfg<NL, F, H, CINR_F16>>>(what, m, a, s);
        case CINR_BF16X3: return launch_all<InrEngine<EngCfg<NL, F, H, CINR_BF16X3>>>(what, m, a, s);
        default: return hipErrorInvalidValue;
    }
}

bool inr_shape_supported(const InrDev& m) {
    if (m.grid) return true;
    const int NL = m.n_levels, F = m.n_features, H = m.hidden;
    return (NL == 8 && F == 2 && H == 32) || (NL == 16 && F == 2 && H == 64) || (NL == 16 && F == 4 && H == 64) ||
           (NL == 8 && F == 2 && H == 64) || (NL == 16 && F == 2 && H == 32);
}

static hipError_t dispatch(int prec, int what, const InrDev& m, const void* a, hipStream_t s) {
    if (m.grid) return launch_all<GridEngine>(what, m, a, s);
    const int NL = m.n_levels, F = m.n_features, H = m.hidden;
    if (NL == 8 && F == 2 && H == 32) return dispatch_prec<8, 2, 32>(prec, what, m, a, s);
    if (NL == 8 && F == 2 && H == 64) return dispatch_prec<8, 2, 64>(prec, what, m, a, s);
    if (NL == 16 && F == 2 && H == 32) return dispatch_prec<16, 2, 32>(prec, what, m, a, s);
    if (NL == 16 && F == 2 && H == 64) return dispatch_prec<16, 2, 64>(prec, what, m, a, s);
    if (NL == 16 && F == 4 && H == 64) return dispatch_prec<16, 4, 64>(prec, what, m, a, s);
    return hipErrorInvalidValue;
}

hipError_t inr_infer_points(const InrDev& m, const float* pos, int64_t n, float* out, int prec, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    PosSrc src{pos, n};
    LinearDst dst{out};
    const void* a[2] = {&src, &dst};
    return dispatch(prec, 0, m, a, s);
}

hipError_t inr_decode_bricks(const InrDev& m, const CacheGeom& g, const int32_t* reqs, const uint32_t* n_dev,
                             const uint32_t* gate, int32_t n_cap, const int32_t* slots, const BrickOut& out,
                             int prec, hipStream_t s, DecodeShape shape) {
    if (n_cap <= 0) return hipSuccess;
    BrickSrc src;
    src.reqs = reqs;
    src.n_dev = n_dev;
    src.gate = gate;
    src.n_host = n_cap;
    src.B = g.brick;
    src.B3 = g.brick * g.brick * g.brick;
    src.n_lods = g.n_lods;
    for (int L = 0; L < kMaxLods; ++L)
        for (int a = 0; a < 3; ++a) src.nb[L][a] = L < g.n_lods ? g.lod[L].nb[a] : 0;
    for (int a = 0; a < 3; ++a) src.dims[a] = m.dims[a];
    BrickDst dst{out.out, out.out16, slots, src.B3, out.split};
    if (shape.parts > 0 && g.brick <= kTabB && g.brick % shape.parts == 0) {
        const int32_t sh[2] = {shape.parts, shape.stage_floats};
        const void* a[3] = {&src, &dst, sh};
        return dispatch(prec, 5, m, a, s);
    }
    const void* a[2] = {&src, &dst};
    return dispatch(prec, 1, m, a, s);
}

hipError_t inr_decode_bricks_multi(const InrDev* d_vols, const InrDev& shape, const CacheGeom& g, const int32_t* reqs,
                                   const int32_t* vols, const uint32_t* n_dev, const uint32_t* gate, int32_t n_cap,
                                   const int32_t* slots, const BrickOut& out, int prec, hipStream_t s,
                                   DecodeShape ds) {
    if (n_cap <= 0) return hipSuccess;
    BrickSrc src;
    src.reqs = reqs;
    src.n_dev = n_dev;
    src.gate = gate;
    src.n_host = n_cap;
    src.B = g.brick;
    src.B3 = g.brick * g.brick * g.brick;
    src.n_lods = g.n_lods;
    for (int L = 0; L < kMaxLods; ++L)
        for (int a = 0; a < 3; ++a) src.nb[L][a] = L < g.n_lods ? g.lod[L].nb[a] : 0;
    for (int a = 0; a < 3; ++a) src.dims[a] = shape.dims[a];
    BrickDst dst{out.out, out.out16, slots, src.B3, out.split};
    if (!shape.grid && ds.parts > 0 && g.brick <= kTabB && g.brick % ds.parts == 0) {
        const int32_t sh[2] = {ds.parts, ds.stage_floats};
        const void* a[5] = {&src, &dst, d_vols, vols, sh};
        return dispatch(prec, 6, shape, a, s);
    }
    const void* a[4] = {&src, &dst, d_vols, vols};
    return dispatch(prec, 4, shape, a, s);
}

hipError_t inr_macrocells(const InrDev& m, int32_t N, float* minmax, int prec, hipStream_t s) {
    int32_t p[4] = {N, (m.dims[0] + N - 1) / N, (m.dims[1] + N - 1) / N, (m.dims[2] + N - 1) / N};
    const void* a[2] = {p, minmax};
    return dispatch(prec, 2, m, a, s);
}

hipError_t inr_infer_misses(const InrDev& m, const float4* rec, const uint32_t* n_dev, int64_t cap, float* vals,
                            int prec, hipStream_t s) {
    MissSrc src{rec, n_dev};
    MissDst dst{rec, vals};
    const void* a[3] = {&src, &dst, &cap};
    return dispatch(prec, 3, m, a, s);
}

}  // namespace cinr
