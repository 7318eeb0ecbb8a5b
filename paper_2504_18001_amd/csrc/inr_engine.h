// INR engine: hash-grid encoding + MLP for one 256-point round of a
// workgroup.  See inr.hip for the data layout.
#pragma once

#include "common.h"

namespace cinr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int NL_, int F_, int H_, int PREC_>
struct EngCfg {
    static constexpr int NL = NL_, F = F_, H = H_, PREC = PREC_;
    static constexpr int IN = NL * F;
    static constexpr int MT = H / 16;  // 16-neuron tiles per hidden layer
};

template <int PREC>
struct Half;
template <>
struct Half<CINR_BF16> {
    typedef __bf16 T;
    typedef bf16x8 V8;
    static constexpr bool kSplit = false;
};
// BF16 with split operands: x = hi + lo (both BF16), products hi*hi + hi*lo
// + lo*hi accumulated in FP32 -- about 16 significant bits per operand.
template <>
struct Half<CINR_BF16X3> {
    typedef __bf16 T;
    typedef bf16x8 V8;
    static constexpr bool kSplit = true;
};
template <>
struct Half<CINR_F16> {
    typedef _Float16 T;
    typedef f16x8 V8;
    static constexpr bool kSplit = false;
};

__device__ inline f32x4 mfma_k32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma_k32(f16x8 a, f16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma_k4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int F>
struct Entry;
template <>
struct Entry<1> {
    __device__ static inline void load(const float* p, float* e) { e[0] = p[0]; }
};
template <>
struct Entry<2> {
    __device__ static inline void load(const float* p, float* e) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        e[0] = v.x;
        e[1] = v.y;
    }
};
template <>
struct Entry<4> {
    __device__ static inline void load(const float* p, float* e) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        e[0] = v.x;
        e[1] = v.y;
        e[2] = v.z;
        e[3] = v.w;
    }
};

// Normalised coordinate u = (clamp(x, 0, V-1) + 0.5) / V in FP64, so that the
// fine levels' cell fractions keep full FP32 precision.
__device__ inline void to_unit(const InrDev& m, const double x[3], double u[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double xa = x[a];
        xa = xa < 0.0 ? 0.0 : xa;
        xa = xa > (double)m.vm1[a] ? (double)m.vm1[a] : xa;
        u[a] = (xa + 0.5) * m.inv_dims[a];
    }
}

// Multi-resolution hash encoding (Section 3) of one level: trilinear
// interpolation of the 8 grid corners around u*N_l.  The level index is
// wave-uniform, so the dense/hashed branch never diverges.
// Cell c = floor(u N_l) and weights w = u N_l - c (FP64, rounded once).
__device__ inline void level_cell(const LevelDev& lv, const double u[3], uint32_t c[3], float w[3]) {
    const double N = lv.res;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double sa = u[a] * N;
        const double fa = floor(sa);
        w[a] = (float)(sa - fa);
        c[a] = (uint32_t)fa;
    }
}

// Table entries of the 8 corners of cell c (x fastest, then y, then z).
__device__ inline void level_corners_idx(const LevelDev& lv, const uint32_t c[3], uint32_t idx[8]) {
    const uint32_t c0 = c[0], c1 = c[1], c2 = c[2];
    if (lv.mask == 0u) {
        const uint32_t sd = lv.side, sd2 = lv.side2;
        const uint32_t b = c0 + c1 * sd + c2 * sd2;
        idx[0] = b;
        idx[1] = b + 1u;
        idx[2] = b + sd;
        idx[3] = b + sd + 1u;
        idx[4] = b + sd2;
        idx[5] = b + sd2 + 1u;
        idx[6] = b + sd2 + sd;
        idx[7] = b + sd2 + sd + 1u;
    } else {
        const uint32_t mk = lv.mask;
        const uint32_t x0 = c0, x1 = c0 + 1u;
        const uint32_t y0 = c1 * kPrime1, y1 = y0 + kPrime1;
        const uint32_t z0 = c2 * kPrime2, z1 = z0 + kPrime2;
        const uint32_t a00 = y0 ^ z0, a10 = y1 ^ z0, a01 = y0 ^ z1, a11 = y1 ^ z1;
        idx[0] = (x0 ^ a00) & mk;
        idx[1] = (x1 ^ a00) & mk;
        idx[2] = (x0 ^ a10) & mk;
        idx[3] = (x1 ^ a10) & mk;
        idx[4] = (x0 ^ a01) & mk;
        idx[5] = (x1 ^ a01) & mk;
        idx[6] = (x0 ^ a11) & mk;
        idx[7] = (x1 ^ a11) & mk;
    }
}

// The 8 corner entries.  The table is under 4 GiB (checked when the volume
// is created), so each load takes the table's uniform base and a 32-bit byte
// offset.
template <int F>
__device__ inline void level_corners_load(const LevelDev& lv, const float* table, const uint32_t idx[8],
                                          float e[8][F]) {
    const char* t8 = reinterpret_cast<const char*>(table);
    const uint32_t b8 = lv.offset * (uint32_t)(F * sizeof(float));
#pragma unroll
    for (int k = 0; k < 8; ++k)
        Entry<F>::load(reinterpret_cast<const float*>(t8 + (b8 + idx[k] * (uint32_t)(F * sizeof(float)))), e[k]);
}

// Trilinear interpolation of the 8 corner entries with weights w.
template <int F>
__device__ inline void level_interp(const float e[8][F], const float w[3], float* out) {
    const float w0 = w[0], w1 = w[1], w2 = w[2];
    const float wx0 = 1.0f - w0, wy0 = 1.0f - w1, wz0 = 1.0f - w2;
    const float wxy[4] = {wx0 * wy0, w0 * wy0, wx0 * w1, w0 * w1};
#pragma unroll
    for (int j = 0; j < F; ++j) out[j] = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float wt = wxy[k & 3] * ((k & 4) ? w2 : wz0);
#pragma unroll
        for (int j = 0; j < F; ++j) out[j] = __builtin_fmaf(wt, e[k][j], out[j]);
    }
}

// The 8 corner entries of cell c from the level's table, interpolated.
template <int F>
__device__ inline void gather_level(const LevelDev& lv, const float* table, const uint32_t c[3], const float w[3],
                                    float* out) {
    uint32_t idx[8];
    level_corners_idx(lv, c, idx);
    float e[8][F];
    level_corners_load<F>(lv, table, idx, e);
    level_interp<F>(e, w, out);
}

template <int F>
__device__ inline void encode_level(const LevelDev& lv, const float* table, const double u[3], float* out) {
    uint32_t c[3];
    float w[3];
    level_cell(lv, u, c, w);
    gather_level<F>(lv, table, c, w, out);
}

// LDS staging of the hash-table corners that the lattice points of one brick
// part touch (brick decoding, Section 4.3.2): per level, the cells of a
// regular block of lattice points span a box of grid corners; a box that fits
// is copied into LDS once, and the part's points interpolate from there.
struct StageLevel {
    int32_t lo[3];  // first corner of the box
    int32_t e[3];   // corners per axis
    int32_t off;    // first float of the box in the stage; -1: read from the table
};

// gather_level for a staged level: the same cell, weights and accumulation
// order, the 8 corners read from the level's box in LDS.
template <int F>
__device__ inline void gather_level_lds(const StageLevel& sl, const float* stage, const uint32_t c[3],
                                        const float w[3], float* out) {
    const float w0 = w[0], w1 = w[1], w2 = w[2];
    const int32_t ex = sl.e[0], exy = sl.e[0] * sl.e[1];
    const int32_t b = ((int32_t)c[0] - sl.lo[0]) + ((int32_t)c[1] - sl.lo[1]) * ex + ((int32_t)c[2] - sl.lo[2]) * exy;
    const int32_t idx[8] = {b, b + 1, b + ex, b + ex + 1, b + exy, b + exy + 1, b + exy + ex, b + exy + ex + 1};
    const float* sp = stage + sl.off;
    float e[8][F];
#pragma unroll
    for (int k = 0; k < 8; ++k) Entry<F>::load(sp + idx[k] * F, e[k]);
    const float wx0 = 1.0f - w0, wy0 = 1.0f - w1, wz0 = 1.0f - w2;
    const float wxy[4] = {wx0 * wy0, w0 * wy0, wx0 * w1, w0 * w1};
#pragma unroll
    for (int j = 0; j < F; ++j) out[j] = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float wt = wxy[k & 3] * ((k & 4) ? w2 : wz0);
#pragma unroll
        for (int j = 0; j < F; ++j) out[j] = __builtin_fmaf(wt, e[k][j], out[j]);
    }
}

// Where a point's per-level cells and weights come from: computed from its
// normalised coordinate, or (brick lattice points, whose coordinates are
// separable) read from per-axis tables that hold the same FP64 results:
// tab[(l * 3 + a) * n + i] = (cell, bits of the weight) of lattice index i
// along axis a at level l.
struct CoordU {
    double u[3];
    __device__ void cell(const LevelDev& lv, int, uint32_t c[3], float w[3]) const { level_cell(lv, u, c, w); }
};
struct CoordTab {
    const uint2* tab;
    int32_t n;
    int32_t i[3];
    __device__ void cell(const LevelDev&, int l, uint32_t c[3], float w[3]) const {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint2 t = tab[(l * 3 + a) * n + i[a]];
            c[a] = t.x;
            w[a] = __uint_as_float(t.y);
        }
    }
};

// Level l of a point: from the stage when its box is there, else from the table.
template <int F, class Coord>
__device__ inline void encode_level_any(const InrDev& m, int l, const Coord& co, const StageLevel* sl,
                                        const float* stage, float* out) {
    uint32_t c[3];
    float w[3];
    co.cell(m.lv[l], l, c, w);
    if (sl && sl[l].off >= 0)
        gather_level_lds<F>(sl[l], stage, c, w, out);
    else
        gather_level<F>(m.lv[l], m.table, c, w, out);
}

__device__ inline float finish_value(const InrDev& m, float y) {
    float v = __builtin_fmaf(m.value_scale, y, m.value_offset);
    v = v < 0.0f ? 0.0f : v;
    v = v > 1.0f ? 1.0f : v;
    return v;
}

// Explicit voxel grid (the fallback source): trilinear interpolation of the
// samples at voxel coordinate x (clamped to [0, V-1]; the last cell is used at
// the upper faces), then the value normalisation.  Same interface as the INR
// engines; no workgroup synchronisation.
struct GridEngine {
    struct Lds {
        int unused;
    };
    __device__ void load_weights(const InrDev&) {}
    __device__ float eval(const InrDev& m, const double x[3], Lds&, const StageLevel* = nullptr,
                          const float* = nullptr) const {
        int32_t j[3];
        float f[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float xa = (float)x[a];
            xa = xa < 0.0f ? 0.0f : (xa > m.vm1[a] ? m.vm1[a] : xa);
            int32_t ja = (int32_t)xa;
            ja = ja > m.dims[a] - 2 ? m.dims[a] - 2 : ja;
            j[a] = ja;
            f[a] = xa - (float)ja;
        }
        const int64_t sy = m.dims[0], sz = (int64_t)m.dims[0] * m.dims[1];
        const float* b = m.grid + j[2] * sz + j[1] * sy + j[0];
        const float c00 = __builtin_fmaf(f[0], b[1] - b[0], b[0]);
        const float c10 = __builtin_fmaf(f[0], b[sy + 1] - b[sy], b[sy]);
        const float c01 = __builtin_fmaf(f[0], b[sz + 1] - b[sz], b[sz]);
        const float c11 = __builtin_fmaf(f[0], b[sz + sy + 1] - b[sz + sy], b[sz + sy]);
        const float c0 = __builtin_fmaf(f[1], c10 - c00, c00);
        const float c1 = __builtin_fmaf(f[1], c11 - c01, c01);
        return finish_value(m, __builtin_fmaf(f[2], c1 - c0, c0));
    }
};

template <class Cfg, bool IS_F32 = (Cfg::PREC == CINR_F32)>
struct InrEngine;

// ---------------------------------------------------------------------------
// FP32 MLP on v_mfma_f32_16x16x4_f32.
// Layer 1, K step (u, r): lane group g supplies feature 16u + 4g + r.
// Layer 2, K step (m', r): lane group g supplies neuron 16m' + 4g + r, which
// is where layer 1's accumulator already holds it.
// ---------------------------------------------------------------------------
template <class Cfg>
struct InrEngine<Cfg, true> {
    static constexpr int NL = Cfg::NL, F = Cfg::F, IN = Cfg::IN, H = Cfg::H, MT = Cfg::MT;
    static constexpr int KU = IN / 16;
    static constexpr int ROW = IN + 4;  // padded row in floats (16-byte aligned)
    static_assert(IN % 16 == 0, "input width must be a multiple of 16");
    struct Lds {
        float f[kBlock * ROW];
    };
    float w1[MT][KU][4];
    float w2[MT][MT][4];
    float w3[MT][4];

    __device__ void load_weights(const InrDev& m) {
        const int lane = threadIdx.x & 63, row = lane & 15, g = lane >> 4;
        const float* W1 = m.weights;
        const float* W2 = W1 + H * IN;
        const float* W3 = W2 + H * H;
#pragma unroll
        for (int t = 0; t < MT; ++t) {
#pragma unroll
            for (int u = 0; u < KU; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) w1[t][u][r] = W1[(16 * t + row) * IN + 16 * u + 4 * g + r];
#pragma unroll
            for (int p = 0; p < MT; ++p)
#pragma unroll
                for (int r = 0; r < 4; ++r) w2[t][p][r] = W2[(16 * t + row) * H + 16 * p + 4 * g + r];
#pragma unroll
            for (int r = 0; r < 4; ++r) w3[t][r] = W3[16 * t + 4 * g + r];
        }
    }

    // All 256 lanes of the workgroup must call eval together.  sl, stage:
    // LDS-staged corner boxes of the levels (brick decoding), or null.
    __device__ float eval(const InrDev& m, const double x[3], Lds& lds, const StageLevel* sl = nullptr,
                          const float* stage = nullptr) {
        CoordU co;
        to_unit(m, x, co.u);
        return eval_c(m, co, lds, sl, stage);
    }

    template <class Coord>
    __device__ float eval_c(const InrDev& m, const Coord& co, Lds& lds, const StageLevel* sl, const float* stage) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, row = lane & 15, g = lane >> 4;
        float* my = lds.f + threadIdx.x * ROW;
        // one level at a time: the FP32 engine's registers leave no room for
        // a second level's corners in flight
#pragma unroll 2
        for (int l = 0; l < NL; ++l) {
            float f[F];
            encode_level_any<F>(m, l, co, sl, stage, f);
#pragma unroll
            for (int j = 0; j < F; ++j) my[l * F + j] = f[j];
        }
        __syncthreads();
        float my_y = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float* pr = lds.f + (wave * 64 + 16 * t + row) * ROW;
            f32x4 h1[MT];
#pragma unroll
            for (int i = 0; i < MT; ++i) h1[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int uu = 0; uu < KU; ++uu) {
                const float4 b = *reinterpret_cast<const float4*>(pr + 16 * uu + 4 * g);
                const float bb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int i = 0; i < MT; ++i) h1[i] = mfma_k4(w1[i][uu][r], bb[r], h1[i]);
            }
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) h1[i][r] = h1[i][r] > 0.0f ? h1[i][r] : 0.0f;
            f32x4 h2[MT];
#pragma unroll
            for (int i = 0; i < MT; ++i) h2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int p = 0; p < MT; ++p)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int i = 0; i < MT; ++i) h2[i] = mfma_k4(w2[i][p][r], h1[p][r], h2[i]);
            float part = 0.0f;
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) part = __builtin_fmaf(w3[i][r], h2[i][r] > 0.0f ? h2[i][r] : 0.0f, part);
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            if (g == t) my_y = part;
        }
        __syncthreads();
        return finish_value(m, my_y);
    }
};

// ---------------------------------------------------------------------------
// BF16 / FP16 MLP on v_mfma_f32_16x16x32_{bf16,f16}, FP32 accumulation; the
// output layer stays FP32.
// Layer 1, K chunk c: lane group g supplies features 32c + 8g + j (zero past
// the input width).  Layer 2, K chunk c: element j of lane group g is neuron
// 32c + 16(j/4) + 4g + j%4, i.e. accumulator tiles 2c and 2c+1.
// ---------------------------------------------------------------------------
template <class Cfg>
struct InrEngine<Cfg, false> {
    static constexpr int NL = Cfg::NL, F = Cfg::F, IN = Cfg::IN, H = Cfg::H, MT = Cfg::MT;
    typedef typename Half<Cfg::PREC>::T T;
    typedef typename Half<Cfg::PREC>::V8 V8;
    static constexpr bool SPLIT = Half<Cfg::PREC>::kSplit;
    static constexpr int NP = SPLIT ? 2 : 1;  // operand parts (hi, lo)
    static constexpr int KC = (IN + 31) / 32;
    static constexpr int KC2 = H / 32;
    static constexpr int ROW = KC * 32 + 8;  // padded row in 16-bit elements (16-byte aligned)
    static_assert(H % 32 == 0, "hidden width must be a multiple of 32");
    struct Lds {
        T f[NP][kBlock * ROW];
    };
    V8 w1[NP][MT][KC];
    V8 w2[NP][MT][KC2];
    float w3[MT][4];

    // x = hi + lo with both parts representable in T
    __device__ static inline T part_hi(float x) { return (T)x; }
    __device__ static inline T part_lo(float x) { return (T)(x - (float)(T)x); }

    __device__ void load_weights(const InrDev& m) {
        const int lane = threadIdx.x & 63, row = lane & 15, g = lane >> 4;
        const float* W1 = m.weights;
        const float* W2 = W1 + H * IN;
        const float* W3 = W2 + H * H;
#pragma unroll
        for (int t = 0; t < MT; ++t) {
#pragma unroll
            for (int c = 0; c < KC; ++c)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = 32 * c + 8 * g + j;
                    const float x = k < IN ? W1[(16 * t + row) * IN + k] : 0.0f;
                    w1[0][t][c][j] = part_hi(x);
                    if (SPLIT) w1[NP - 1][t][c][j] = part_lo(x);
                }
#pragma unroll
            for (int c = 0; c < KC2; ++c)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float x = W2[(16 * t + row) * H + 32 * c + 16 * (j >> 2) + 4 * g + (j & 3)];
                    w2[0][t][c][j] = part_hi(x);
                    if (SPLIT) w2[NP - 1][t][c][j] = part_lo(x);
                }
#pragma unroll
            for (int r = 0; r < 4; ++r) w3[t][r] = W3[16 * t + 4 * g + r];
        }
    }

    __device__ float eval(const InrDev& m, const double x[3], Lds& lds, const StageLevel* sl = nullptr,
                          const float* stage = nullptr) {
        CoordU co;
        to_unit(m, x, co.u);
        return eval_c(m, co, lds, sl, stage);
    }

    template <class Coord>
    __device__ float eval_c(const InrDev& m, const Coord& co, Lds& lds, const StageLevel* sl, const float* stage) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, row = lane & 15, g = lane >> 4;
        T* my = lds.f[0] + threadIdx.x * ROW;
        T* my_lo = lds.f[NP - 1] + threadIdx.x * ROW;
#pragma unroll 2
        for (int l = 0; l < NL; ++l) {
            float f[F];
            encode_level_any<F>(m, l, co, sl, stage, f);
#pragma unroll
            for (int j = 0; j < F; ++j) {
                my[l * F + j] = part_hi(f[j]);
                if (SPLIT) my_lo[l * F + j] = part_lo(f[j]);
            }
        }
        // zero padding of the K chunk past the input width
#pragma unroll
        for (int k = IN; k < KC * 32; ++k) {
            my[k] = (T)0.0f;
            my_lo[k] = (T)0.0f;
        }
        __syncthreads();
        float my_y = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int pr = (wave * 64 + 16 * t + row) * ROW;
            f32x4 h1[MT];
#pragma unroll
            for (int i = 0; i < MT; ++i) h1[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const V8 b = *reinterpret_cast<const V8*>(lds.f[0] + pr + 32 * c + 8 * g);
#pragma unroll
                for (int i = 0; i < MT; ++i) h1[i] = mfma_k32(w1[0][i][c], b, h1[i]);
                if (SPLIT) {
                    const V8 bl = *reinterpret_cast<const V8*>(lds.f[NP - 1] + pr + 32 * c + 8 * g);
#pragma unroll
                    for (int i = 0; i < MT; ++i) {
                        h1[i] = mfma_k32(w1[0][i][c], bl, h1[i]);
                        h1[i] = mfma_k32(w1[NP - 1][i][c], b, h1[i]);
                    }
                }
            }
            f32x4 h2[MT];
#pragma unroll
            for (int i = 0; i < MT; ++i) h2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < KC2; ++c) {
                V8 b, bl = {};
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    float h = h1[2 * c + (j >> 2)][j & 3];
                    h = h > 0.0f ? h : 0.0f;
                    b[j] = part_hi(h);
                    if (SPLIT) bl[j] = part_lo(h);
                }
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    h2[i] = mfma_k32(w2[0][i][c], b, h2[i]);
                    if (SPLIT) {
                        h2[i] = mfma_k32(w2[0][i][c], bl, h2[i]);
                        h2[i] = mfma_k32(w2[NP - 1][i][c], b, h2[i]);
                    }
                }
            }
            float part = 0.0f;
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) part = __builtin_fmaf(w3[i][r], h2[i][r] > 0.0f ? h2[i][r] : 0.0f, part);
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            if (g == t) my_y = part;
        }
        __syncthreads();
        return finish_value(m, my_y);
    }
};

}  // namespace cinr
