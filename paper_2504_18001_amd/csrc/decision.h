// Decision plane of the sampler: ray setup, sample positions, stochastic LoD
// and page-table addressing.  Every expression is a single correctly rounded
// binary32 operation (the library is compiled with -ffp-contract=off, FP32
// division and square root are correctly rounded), so these decisions are
// reproducible bit for bit by any IEEE implementation of the same sequence.
#pragma once

#include "common.h"

namespace cinr {

struct CamDev {
    int32_t proj, W, H;
    float eye[3], fwd[3], right[3], up[3];
    float tanx, tany, ow, oh;
};

// Primary ray through the centre of pixel (i, j) (row 0 at the top) and its
// parametric overlap [ts, te] with the box [0, V-1]^3 (slab test).
// kOFirst only orders the stores of the perspective branch (o before d, as
// the orthographic branch): the path tracer keeps its o and d in registers
// that way, while the ray marcher's register allocation prefers d first.
template <bool kOFirst = false>
__device__ inline bool ray_setup(const CamDev& c, const float vm1[3], int32_t i, int32_t j, float o[3], float d[3],
                                 float& ts, float& te) {
    const float fx = ((float)i + 0.5f) / (float)c.W;
    const float fy = ((float)j + 0.5f) / (float)c.H;
    if (c.proj == CINR_PERSPECTIVE) {
        const float sx = (fx * 2.0f - 1.0f) * c.tanx;
        const float sy = (1.0f - fy * 2.0f) * c.tany;
        float dir[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float r = sx * c.right[a];
            const float s = c.fwd[a] + r;
            const float u = sy * c.up[a];
            dir[a] = s + u;
        }
        float n2 = dir[0] * dir[0];
        const float y2 = dir[1] * dir[1];
        const float z2 = dir[2] * dir[2];
        n2 = n2 + y2;
        n2 = n2 + z2;
        const float n = __builtin_sqrtf(n2);
        if constexpr (kOFirst) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                o[a] = c.eye[a];
                d[a] = dir[a] / n;
            }
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                d[a] = dir[a] / n;
                o[a] = c.eye[a];
            }
        }
    } else {
        const float ox = (fx - 0.5f) * c.ow;
        const float oy = (0.5f - fy) * c.oh;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float r = ox * c.right[a];
            const float s = c.eye[a] + r;
            const float u = oy * c.up[a];
            o[a] = s + u;
            d[a] = c.fwd[a];
        }
    }
    float tlo = -__builtin_inff(), thi = __builtin_inff();
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) {
            if (o[a] < 0.0f || o[a] > vm1[a]) inside = false;
        } else {
            const float ta = (0.0f - o[a]) / d[a];
            const float tb = (vm1[a] - o[a]) / d[a];
            const float lo = ta < tb ? ta : tb;
            const float hi = ta < tb ? tb : ta;
            if (lo > tlo) tlo = lo;
            if (hi < thi) thi = hi;
        }
    }
    const float t0 = tlo > 0.0f ? tlo : 0.0f;
    ts = t0;
    te = thi;
    // a degenerate direction leaves the exit at infinity: no samples
    return inside && (thi >= t0) && (thi < __builtin_inff());
}

// Sample k of a ray: t = ts + k*step (false past te); position clamped to the box.
__device__ inline bool sample_pos(const float o[3], const float d[3], float ts, float te, float step, int32_t k,
                                  const float vm1[3], float p[3]) {
    const float kk = (float)k * step;
    const float t = ts + kk;
    if (t > te) return false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float td = t * d[a];
        float q = o[a] + td;
        if (q < 0.0f) q = 0.0f;
        if (q > vm1[a]) q = vm1[a];
        p[a] = q;
    }
    return true;
}

// Step exponent of a macro-cell of maximum opacity mu > 0 under the adaptive
// sampling rate (Section 5.2): min(E, floor(-log2 mu)), 0 for mu >= 1, from
// the binary32 fields (mu = m 2^x with m in [1, 2): -log2 mu is in
// (-x - 1, -x], equal to -x when m = 1).
__device__ inline int32_t step_exp(float mu, int32_t E) {
    if (mu >= 1.0f) return 0;
    const uint32_t bits = __float_as_uint(mu);
    const int32_t x = (int32_t)((bits >> 23) & 0xFFu) - 127;
    const int32_t e = (bits & 0x7FFFFFu) == 0u ? -x : -x - 1;
    return e < E ? e : E;
}

__device__ inline uint32_t xorshift32(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

// Stochastic LoD (Algorithm 2, Section 5.3): D = |p - eye| * lod_scale; the
// integer part of D, one level coarser when a uniform variate from xorshift
// of (bits of D) XOR (frame seed) is below the fractional part; clamped to
// [lod_floor, n_lods - 1].
__device__ inline int32_t select_lod(const float p[3], const float eye[3], float lod_scale, float factor,
                                     uint32_t frame_seed, int32_t lod_floor, int32_t n_lods) {
    const float dx = p[0] - eye[0];
    const float dy = p[1] - eye[1];
    const float dz = p[2] - eye[2];
    float s = dx * dx;
    const float sy = dy * dy;
    const float sz = dz * dz;
    s = s + sy;
    s = s + sz;
    const float D0 = __builtin_sqrtf(s) * lod_scale;
    const float D = D0 * factor;  // context-aware LoD (1 otherwise)
    const float fl = __builtin_floorf(D);
    const float fr = D - fl;
    const uint32_t r = xorshift32(__float_as_uint(D) ^ frame_seed);
    const float u = (float)(r >> 8) * 5.9604644775390625e-08f;  // 2^-24
    int32_t L;
    if (fl >= (float)(n_lods - 1)) {
        L = n_lods - 1;
    } else {
        L = (int32_t)fl;
        if (u < fr) L += 1;
    }
    if (L < lod_floor) L = lod_floor;
    if (L > n_lods - 1) L = n_lods - 1;
    return L;
}

// Brick of LoD L holding sample position p: lattice cell j (clamped so that
// j+1 exists), brick b = j / (B-1), key, and the cell fraction q - j.  Keys
// fit in 31 bits (checked when the cache is created).
struct BrickAddr {
    int32_t key;
    int32_t lj[3];   // cell inside the brick (j - b(B-1))
    float frac[3];
};

// `lg` is the geometry of LoD L; kB is the brick size when it is known at
// compile time (0: `brick`, with `div_b1` dividing by brick - 1).
template <int kB>
__device__ inline BrickAddr brick_addr(const LodGeom& lg, int32_t brick, FastDiv div_b1, int32_t L, const float p[3]) {
    BrickAddr r;
    const float sc = __builtin_ldexpf(1.0f, -L);
    const int32_t B1 = (kB ? kB : brick) - 1;
    int32_t b[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float q = p[a] * sc;
        int32_t j = (int32_t)q;
        if (j > lg.K[a] - 2) j = lg.K[a] - 2;
        b[a] = kB ? (int32_t)((uint32_t)j / (uint32_t)(kB - 1)) : (int32_t)fast_div((uint32_t)j, div_b1);
        r.lj[a] = j - b[a] * B1;
        r.frac[a] = q - (float)j;
    }
    r.key = (int32_t)lg.off + (b[2] * lg.nb[1] + b[1]) * lg.nb[0] + b[0];
    return r;
}

// The brick of LoD L holding p (coordinates b) and its key alone: the same
// operations as brick_addr, for the page-table search over the LoDs.
template <int kB>
__device__ inline int32_t brick_key(const LodGeom& lg, int32_t brick, FastDiv div_b1, int32_t L, const float p[3],
                                    int32_t b[3]) {
    const float sc = __builtin_ldexpf(1.0f, -L);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float q = p[a] * sc;
        int32_t j = (int32_t)q;
        if (j > lg.K[a] - 2) j = lg.K[a] - 2;
        b[a] = kB ? (int32_t)((uint32_t)j / (uint32_t)(kB - 1)) : (int32_t)fast_div((uint32_t)j, div_b1);
    }
    (void)brick;
    return (int32_t)lg.off + (b[2] * lg.nb[1] + b[1]) * lg.nb[0] + b[0];
}

// Path tracing draws (Section 5.1; binary32 decision plane).
// A uniform in [0, 1) from the top 24 bits of a random word.
__device__ inline float pt_uniform(uint32_t r) { return (float)(r >> 8) * 5.9604644775390625e-08f; }

// Free-flight length in units of 1 / majorant: -ln(xi), xi = ((r >> 8) + 1)
// 2^-24 in (0, 1], the logarithm in binary64 rounded once to binary32.
__device__ inline float pt_free_flight(uint32_t r) {
    const double xi = ((double)(r >> 8) + 1.0) * 5.9604644775390625e-08;
    return (float)(-log(xi));
}

// Marsaglia (1972): (u1, u2) uniform in [-1, 1)^2, accepted when
// s = u1^2 + u2^2 is in (0, 1); then (2 u1 sqrt(1-s), 2 u2 sqrt(1-s), 1-2s)
// is uniform on the unit sphere.
__device__ inline bool pt_marsaglia(const uint32_t r[4], float d[3]) {
    const float u1 = 2.0f * pt_uniform(r[0]) - 1.0f;
    const float u2 = 2.0f * pt_uniform(r[1]) - 1.0f;
    const float a = u1 * u1;
    const float b = u2 * u2;
    const float s = a + b;
    if (s >= 1.0f || s == 0.0f) return false;
    const float q = __builtin_sqrtf(1.0f - s);
    d[0] = (2.0f * u1) * q;
    d[1] = (2.0f * u2) * q;
    d[2] = 1.0f - 2.0f * s;
    return true;
}

// Distance from p (in the box [0, vm1]) along d to the box boundary.
__device__ inline float pt_segment_exit(const float p[3], const float d[3], const float vm1[3]) {
    float t = __builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) continue;
        const float wall = d[a] > 0.0f ? vm1[a] : 0.0f;
        const float ta = (wall - p[a]) / d[a];
        if (ta < t) t = ta;
    }
    if (!(t >= 0.0f) || t == __builtin_inff()) t = 0.0f;
    return t;
}

// Position o + t d, clamped to the box.
__device__ inline void pt_pos(const float o[3], const float d[3], float t, const float vm1[3], float p[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float td = t * d[a];
        float q = o[a] + td;
        if (q < 0.0f) q = 0.0f;
        if (q > vm1[a]) q = vm1[a];
        p[a] = q;
    }
}

}  // namespace cinr
