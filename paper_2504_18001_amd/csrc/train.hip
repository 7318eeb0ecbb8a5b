// Training of the hash-grid INR on gfx950 (the learned part): MSE of the raw
// MLP output against an explicit grid at uniform points (Section 4.1 fits
// the INR to the data), analytic backward through MLP and hash grid, Adam.
//
// k_train_grad is persistent; each wave takes tiles of P = 32 points:
//  - every lane encodes half of the levels of one point into LDS, both as
//    rows (point-major) and as columns (feature-major);
//  - the MLP forward and backward products run on MFMA (16x16x32 BF16 or
//    16x16x4 FP32) over LDS tiles whose K index is contiguous for both
//    operands; activations and their gradients are staged in both layouts so
//    that the weight gradients (a contraction over points) use the same
//    helper;
//  - weight gradients accumulate in registers per wave and are written once
//    as a per-wave partial, summed by k_train_reduce (fixed order);
//  - the feature gradient of every point is scattered into the table
//    gradient with FP32 atomics (8 corners x F features per level).
#include "frame.h"
#include "inr_engine.h"

namespace cinr {

namespace {

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// D (16x16, lane l: rows 4*(l/16)+r of column l%16) += A * B over K, with A
// row-major (16 rows, stride lda) and B given as B^T row-major (16 rows =
// columns of B, stride ldb); K is contiguous in both, in LDS.
template <int PREC>
struct Mma;
template <>
struct Mma<CINR_BF16> {
    typedef __bf16 T;
    __device__ static f32x4 tile(const T* A, int lda, const T* BT, int ldb, int K, f32x4 acc) {
        const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
        for (int k0 = 0; k0 < K; k0 += 32) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(A + r * lda + k0 + 8 * g);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(BT + r * ldb + k0 + 8 * g);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
        return acc;
    }
};
template <>
struct Mma<CINR_F32> {
    typedef float T;
    __device__ static f32x4 tile(const T* A, int lda, const T* BT, int ldb, int K, f32x4 acc) {
        const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
        for (int k0 = 0; k0 < K; k0 += 4)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[r * lda + k0 + g], BT[r * ldb + k0 + g], acc, 0, 0, 0);
        return acc;
    }
};

// Corner indices and trilinear weights of one level at u (the forward
// encoding of encode_level, kept for the scatter of the backward pass).
__device__ inline void level_corners(const LevelDev& lv, const double u[3], uint32_t idx[8], float wt[8]) {
    const double N = lv.res;
    const double s0 = u[0] * N, s1 = u[1] * N, s2 = u[2] * N;
    const double f0 = floor(s0), f1 = floor(s1), f2 = floor(s2);
    const float w0 = (float)(s0 - f0), w1 = (float)(s1 - f1), w2 = (float)(s2 - f2);
    const uint32_t c0 = (uint32_t)f0, c1 = (uint32_t)f1, c2 = (uint32_t)f2;
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
    const float wx0 = 1.0f - w0, wy0 = 1.0f - w1, wz0 = 1.0f - w2;
    const float wxy[4] = {wx0 * wy0, w0 * wy0, wx0 * w1, w0 * w1};
#pragma unroll
    for (int k = 0; k < 8; ++k) wt[k] = wxy[k & 3] * ((k & 4) ? w2 : wz0);
}

}  // namespace

// LDS layout of the gradient kernel for one architecture and precision.
template <class Cfg, int PREC>
struct TrainShape {
    typedef typename Mma<PREC>::T T;
    static constexpr int NL = Cfg::NL, F = Cfg::F, IN = Cfg::IN, H = Cfg::H;
    static constexpr int P = 32;                    // points per wave tile
    static constexpr int KI = (IN + 31) / 32 * 32;  // input width padded for the MFMA K step
    static constexpr int PAD = 16 / (int)sizeof(T); // 16 bytes of row padding
    static constexpr int LX = KI + PAD;             // rows with K = inputs
    static constexpr int LH = H + PAD;              // rows with K = neurons
    static constexpr int LP = P + PAD;              // rows with K = points
    static constexpr int LDX = KI + 4;              // f32 feature-gradient rows
    // weights: W1 [H][KI], W1^T [KI][H], W2 [H][H], W2^T [H][H] (element type T), W3 [H] (f32)
    static constexpr int W_ELEMS = H * LX + KI * LH + 2 * H * LH;
    static constexpr int W_BYTES = (W_ELEMS * (int)sizeof(T) + H * 4 + 15) / 16 * 16;
    // per wave: X, X^T, A1, A1^T, dZ2, dZ2^T (T).  dZ1 overwrites A1 in place
    // (each lane reads the mask and writes the gradient of the same
    // elements), dX (f32) reuses the dZ2 area once dZ2 is consumed.
    static constexpr int V_ELEMS = P * LX + KI * LP + 2 * (P * LH + H * LP);
    static constexpr int V_BYTES = (V_ELEMS * (int)sizeof(T) + 15) / 16 * 16;
    static_assert(P * LDX * 4 <= (P * LH + H * LP) * (int)sizeof(T), "dX does not fit in the dZ2 area");
    static constexpr int kLdsMax = 160 * 1024;
    static constexpr int WAVES_FIT = (kLdsMax - W_BYTES) / V_BYTES;
    static constexpr int WAVES = WAVES_FIT >= 4 ? 4 : (WAVES_FIT >= 2 ? 2 : 1);
    static constexpr int LDS = W_BYTES + WAVES * V_BYTES;
    // the rest of the LDS accumulates the table gradient of the leading dense
    // (coarse) levels, whose few entries every point touches
    static constexpr int ACC_FLOATS = (kLdsMax - LDS) / 4;
    static constexpr int NW = H * IN + H * H + H;  // MLP weights
    static_assert(H % 32 == 0, "hidden width must be a multiple of 32");
    static_assert(WAVES_FIT >= 1, "training tile does not fit in LDS");
};

struct TrainArgs {
    const float* u;       // [n][3] points in [0,1)^3
    const float* target;  // [n]
    int64_t n;
    float scale;          // d loss / d y = scale * (y - target)
    float* g_table;       // [entries][F], accumulated with atomics
    float* partial;       // [waves][NW + 1]: weight gradients and loss of each wave
    int32_t lds_levels;   // levels [0, lds_levels) are accumulated in LDS first
    int32_t lds_floats;   // their gradient entries (entries * F), <= ACC_FLOATS
};

template <class Cfg, int PREC>
__global__ __launch_bounds__(256) void k_train_grad(InrDev m, TrainArgs a) {
    using S = TrainShape<Cfg, PREC>;
    using T = typename S::T;
    constexpr int NL = S::NL, F = S::F, IN = S::IN, H = S::H, P = S::P, KI = S::KI;
    constexpr int LX = S::LX, LH = S::LH, LP = S::LP, LDX = S::LDX, MTH = H / 16, MTI = (IN + 15) / 16;
    __shared__ __attribute__((aligned(16))) char smem[S::LDS];
    __shared__ float sAcc[S::ACC_FLOATS > 0 ? S::ACC_FLOATS : 1];
    T* sW1 = reinterpret_cast<T*>(smem);
    T* sW1T = sW1 + H * LX;
    T* sW2 = sW1T + KI * LH;
    T* sW2T = sW2 + H * LH;
    float* sW3 = reinterpret_cast<float*>(sW2T + H * LH);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    char* vbase = smem + S::W_BYTES + wave * S::V_BYTES;
    T* sX = reinterpret_cast<T*>(vbase);
    T* sXT = sX + P * LX;
    T* sA1 = sXT + KI * LP;
    T* sA1T = sA1 + P * LH;
    T* sD2 = sA1T + H * LP;
    T* sD2T = sD2 + P * LH;
    T* sD1 = sA1;
    T* sD1T = sA1T;
    float* sDX = reinterpret_cast<float*>(sD2);

    // weights (zero past the input width), in both layouts
    const float* W1 = m.weights;
    const float* W2 = W1 + H * IN;
    const float* W3 = W2 + H * H;
    for (int e = threadIdx.x; e < H * KI; e += blockDim.x) {
        const int n = e / KI, i = e % KI;
        const T v = (T)(i < IN ? W1[n * IN + i] : 0.0f);
        sW1[n * LX + i] = v;
        sW1T[i * LH + n] = v;
    }
    for (int e = threadIdx.x; e < H * H; e += blockDim.x) {
        const int n = e / H, k = e % H;
        const T v = (T)W2[e];
        sW2[n * LH + k] = v;
        sW2T[k * LH + n] = v;
    }
    for (int e = threadIdx.x; e < H; e += blockDim.x) sW3[e] = W3[e];
    for (int e = threadIdx.x; e < a.lds_floats; e += blockDim.x) sAcc[e] = 0.0f;
    // the padded input columns of X stay zero
    if constexpr (KI > IN) {
        for (int e = lane; e < P * (KI - IN); e += 64) {
            const int q = e / (KI - IN), i = IN + e % (KI - IN);
            sX[q * LX + i] = (T)0.0f;
            sXT[i * LP + q] = (T)0.0f;
        }
    }
    __syncthreads();

    f32x4 gw1[MTH][MTI], gw2[MTH][MTH];
#pragma unroll
    for (int i = 0; i < MTH; ++i) {
#pragma unroll
        for (int j = 0; j < MTI; ++j) gw1[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < MTH; ++j) gw2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gw3[MTH];
#pragma unroll
    for (int i = 0; i < MTH; ++i) gw3[i] = 0.0f;
    float loss = 0.0f;

    const int64_t n_tiles = (a.n + P - 1) / P;
    const int64_t wave_g = (int64_t)blockIdx.x * S::WAVES + wave;
    const int64_t n_waves = (int64_t)gridDim.x * S::WAVES;
    const int q = lane & (P - 1), half = lane >> 5;  // encoding: point q, levels of one half
    constexpr int L0 = 0, L1 = NL / 2;
    for (int64_t tile = wave_g; tile < n_tiles; tile += n_waves) {
        const int64_t p0 = tile * P;
        // ---- encode
        {
            const int64_t pi = p0 + q;
            const bool ok = pi < a.n;
            double u[3] = {0.5, 0.5, 0.5};
            if (ok) {
                u[0] = a.u[3 * pi];
                u[1] = a.u[3 * pi + 1];
                u[2] = a.u[3 * pi + 2];
            }
            const int lb = half ? L1 : L0, le = half ? NL : L1;
            for (int l = lb; l < le; ++l) {
                float f[F];
                encode_level<F>(m.lv[l], m.table, u, f);
#pragma unroll
                for (int j = 0; j < F; ++j) {
                    const T v = (T)(ok ? f[j] : 0.0f);
                    sX[q * LX + l * F + j] = v;
                    sXT[(l * F + j) * LP + q] = v;
                }
            }
        }
        wave_sync();
        // ---- layer 1: Z1 = X W1^T, A1 = relu(Z1)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < MTH; ++nt) {
                f32x4 z = Mma<PREC>::tile(sX + 16 * mt * LX, LX, sW1 + 16 * nt * LX, LX, KI, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int pt = 16 * mt + 4 * g + r, n = 16 * nt + c;
                    const T v = (T)(z[r] > 0.0f ? z[r] : 0.0f);
                    sA1[pt * LH + n] = v;
                    sA1T[n * LP + pt] = v;
                }
            }
        wave_sync();
        // ---- layer 2: Z2 = A1 W2^T; output y = W3 relu(Z2); dZ2 = dy W3 [Z2 > 0]
        f32x4 z2[2][MTH];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < MTH; ++nt)
                z2[mt][nt] = Mma<PREC>::tile(sA1 + 16 * mt * LH, LH, sW2 + 16 * nt * LH, LH, H, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int nt = 0; nt < MTH; ++nt) {
                const float w3 = sW3[16 * nt + c];
#pragma unroll
                for (int r = 0; r < 4; ++r) part[r] = __builtin_fmaf(w3, z2[mt][nt][r] > 0.0f ? z2[mt][nt][r] : 0.0f, part[r]);
            }
            // sum over the 16 columns of the group
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) part[r] += __shfl_xor(part[r], o);
            float dy[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t pi = p0 + 16 * mt + 4 * g + r;
                const bool ok = pi < a.n;
                const float e = ok ? part[r] - a.target[pi] : 0.0f;
                if (c == 0) loss = __builtin_fmaf(e, e, loss);
                dy[r] = a.scale * e;
            }
#pragma unroll
            for (int nt = 0; nt < MTH; ++nt) {
                const int n = 16 * nt + c;
                const float w3 = sW3[n];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float zz = z2[mt][nt][r];
                    const int pt = 16 * mt + 4 * g + r;
                    gw3[nt] = __builtin_fmaf(dy[r], zz > 0.0f ? zz : 0.0f, gw3[nt]);
                    const T d = (T)(zz > 0.0f ? dy[r] * w3 : 0.0f);
                    sD2[pt * LH + n] = d;
                    sD2T[n * LP + pt] = d;
                }
            }
        }
        wave_sync();
        // ---- dW2 += dZ2^T A1
#pragma unroll
        for (int nt = 0; nt < MTH; ++nt)
#pragma unroll
            for (int kt = 0; kt < MTH; ++kt)
                gw2[nt][kt] = Mma<PREC>::tile(sD2T + 16 * nt * LP, LP, sA1T + 16 * kt * LP, LP, P, gw2[nt][kt]);
        // ---- dZ1 = (dZ2 W2) [A1 > 0]
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int kt = 0; kt < MTH; ++kt) {
                f32x4 d = Mma<PREC>::tile(sD2 + 16 * mt * LH, LH, sW2T + 16 * kt * LH, LH, H, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int pt = 16 * mt + 4 * g + r, k = 16 * kt + c;
                    const T v = (T)((float)sA1[pt * LH + k] > 0.0f ? d[r] : 0.0f);
                    sD1[pt * LH + k] = v;
                    sD1T[k * LP + pt] = v;
                }
            }
        wave_sync();
        // ---- dW1 += dZ1^T X; dX = dZ1 W1
#pragma unroll
        for (int nt = 0; nt < MTH; ++nt)
#pragma unroll
            for (int it = 0; it < MTI; ++it)
                gw1[nt][it] = Mma<PREC>::tile(sD1T + 16 * nt * LP, LP, sXT + 16 * it * LP, LP, P, gw1[nt][it]);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int it = 0; it < MTI; ++it) {
                f32x4 d = Mma<PREC>::tile(sD1 + 16 * mt * LH, LH, sW1T + 16 * it * LH, LH, H, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int r = 0; r < 4; ++r) sDX[(16 * mt + 4 * g + r) * LDX + 16 * it + c] = d[r];
            }
        wave_sync();
        // ---- scatter of the feature gradient into the table gradient
        {
            const int64_t pi = p0 + q;
            if (pi < a.n) {
                const double u[3] = {a.u[3 * pi], a.u[3 * pi + 1], a.u[3 * pi + 2]};
                const int lb = half ? L1 : L0, le = half ? NL : L1;
                for (int l = lb; l < le; ++l) {
                    uint32_t idx[8];
                    float wt[8];
                    level_corners(m.lv[l], u, idx, wt);
                    float dxf[F];
#pragma unroll
                    for (int j = 0; j < F; ++j) dxf[j] = sDX[q * LDX + l * F + j];
                    if (l < a.lds_levels) {
                        float* gt = sAcc + m.lv[l].offset * F;
#pragma unroll
                        for (int k = 0; k < 8; ++k)
#pragma unroll
                            for (int j = 0; j < F; ++j) atomicAdd(gt + idx[k] * F + j, wt[k] * dxf[j]);
                    } else {
                        float* gt = a.g_table + (size_t)m.lv[l].offset * F;
#pragma unroll
                        for (int k = 0; k < 8; ++k)
#pragma unroll
                            for (int j = 0; j < F; ++j) atomicAdd(gt + (size_t)idx[k] * F + j, wt[k] * dxf[j]);
                    }
                }
            }
        }
        wave_sync();
    }

    // ---- the block's coarse-level gradients, one atomic per entry
    __syncthreads();
    for (int e = threadIdx.x; e < a.lds_floats; e += blockDim.x) {
        const float v = sAcc[e];
        if (v != 0.0f) atomicAdd(a.g_table + e, v);
    }
    // ---- per-wave partials: W1 [H][IN], W2 [H][H], W3 [H], loss
    float* out = a.partial + wave_g * (S::NW + 1);
#pragma unroll
    for (int nt = 0; nt < MTH; ++nt) {
#pragma unroll
        for (int it = 0; it < MTI; ++it)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * nt + 4 * g + r, i = 16 * it + c;
                if (i < IN) out[n * IN + i] = gw1[nt][it][r];
            }
#pragma unroll
        for (int kt = 0; kt < MTH; ++kt)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[H * IN + (16 * nt + 4 * g + r) * H + 16 * kt + c] = gw2[nt][kt][r];
        float v = gw3[nt];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (g == 0) out[H * IN + H * H + 16 * nt + c] = v;
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) loss += __shfl_xor(loss, o);
    if (lane == 0) out[S::NW] = loss;
}

// Sum of the per-wave partials in a fixed order: out[j] = sum_w partial[w][j]
// (j < nw), loss = sum_w partial[w][nw] / n.
__global__ void k_train_reduce(const float* partial, int64_t n_waves, int32_t nw, float* g_weights, float* loss,
                               float inv_n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > nw) return;
    float s = 0.0f;
    for (int64_t w = 0; w < n_waves; ++w) s += partial[w * (nw + 1) + j];
    if (j < nw)
        g_weights[j] = s;
    else if (loss)
        *loss = s * inv_n;
}

// Training points and targets: Philox-4x32-10 per point, counter (i, step),
// key (seed); 24 bits per coordinate; target = trilinear interpolation of the
// grid at x = clamp(u V - 0.5, 0, V - 1).

__global__ void k_train_points(uint64_t seed, int64_t step, int64_t n, const float* grid, int32_t vx, int32_t vy,
                               int32_t vz, float* u_out, float* target) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)step, (uint32_t)((uint64_t)step >> 32)};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    float u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = (float)(c[a] >> 8) * 5.9604644775390625e-08f;  // 2^-24
    u_out[3 * i] = u[0];
    u_out[3 * i + 1] = u[1];
    u_out[3 * i + 2] = u[2];
    if (!grid) return;
    const int32_t V[3] = {vx, vy, vz};
    int32_t j[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // u has 24 significant bits and V <= 2^24: u*V and the shift are exact
        float x = u[a] * (float)V[a] - 0.5f;
        x = x < 0.0f ? 0.0f : x;
        x = x > (float)(V[a] - 1) ? (float)(V[a] - 1) : x;
        int32_t jj = (int32_t)x;
        jj = jj > V[a] - 2 ? V[a] - 2 : jj;
        jj = jj < 0 ? 0 : jj;
        j[a] = jj;
        f[a] = V[a] > 1 ? x - (float)jj : 0.0f;
    }
    const int64_t sy = vx, sz = (int64_t)vx * vy;
    const int64_t dx = vx > 1 ? 1 : 0, dy = vy > 1 ? sy : 0, dz = vz > 1 ? sz : 0;
    const float* b = grid + j[2] * sz + j[1] * sy + j[0];
    const float c00 = __builtin_fmaf(f[0], b[dx] - b[0], b[0]);
    const float c10 = __builtin_fmaf(f[0], b[dy + dx] - b[dy], b[dy]);
    const float c01 = __builtin_fmaf(f[0], b[dz + dx] - b[dz], b[dz]);
    const float c11 = __builtin_fmaf(f[0], b[dz + dy + dx] - b[dz + dy], b[dz + dy]);
    const float c0 = __builtin_fmaf(f[1], c10 - c00, c00);
    const float c1 = __builtin_fmaf(f[1], c11 - c01, c01);
    target[i] = __builtin_fmaf(f[2], c1 - c0, c0);
}

// Adam (Kingma and Ba 2015) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
// (computed by the host in FP64); the gradient is cleared after use when
// `clear` is set.
__global__ void k_adam(float* p, float* m1, float* m2, float* g, int64_t n, float lr, float b1, float b2, float eps,
                       float inv_c1, float inv_c2, int32_t clear) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float a = __builtin_fmaf(b1, m1[i], (1.0f - b1) * gi);
        const float b = __builtin_fmaf(b2, m2[i], (1.0f - b2) * gi * gi);
        m1[i] = a;
        m2[i] = b;
        p[i] -= lr * (a * inv_c1) / (__builtin_sqrtf(b * inv_c2) + eps);
        if (clear) g[i] = 0.0f;
    }
}

__global__ void k_fill(float* p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <class Cfg, int PREC>
static hipError_t launch_grad_t(const InrDev& m, TrainArgs a, int64_t max_waves, int64_t* waves_used,
                                hipStream_t s) {
    using S = TrainShape<Cfg, PREC>;
    // leading dense levels whose gradient fits in the spare LDS (their table
    // entries start at offset 0 and are contiguous)
    a.lds_levels = 0;
    a.lds_floats = 0;
    for (int l = 0; l < m.n_levels && m.lv[l].mask == 0u; ++l) {
        const int64_t end = ((int64_t)m.lv[l].offset + (int64_t)m.lv[l].side * m.lv[l].side2) * S::F;
        if (end > S::ACC_FLOATS) break;
        a.lds_levels = l + 1;
        a.lds_floats = (int32_t)end;
    }
    const int64_t tiles = (a.n + S::P - 1) / S::P;
    int64_t blocks = (tiles + S::WAVES - 1) / S::WAVES;
    const int64_t cap = max_waves / S::WAVES;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    *waves_used = blocks * S::WAVES;
    hipLaunchKernelGGL((k_train_grad<Cfg, PREC>), dim3((unsigned)blocks), dim3(64 * S::WAVES), 0, s, m, a);
    return hipGetLastError();
}

template <int NL, int F, int H>
static hipError_t launch_grad_p(int prec, const InrDev& m, const TrainArgs& a, int64_t max_waves, int64_t* used,
                                hipStream_t s) {
    if (prec == CINR_BF16) return launch_grad_t<EngCfg<NL, F, H, CINR_BF16>, CINR_BF16>(m, a, max_waves, used, s);
    return launch_grad_t<EngCfg<NL, F, H, CINR_F32>, CINR_F32>(m, a, max_waves, used, s);
}

bool train_shape_supported(const InrDev& m) { return !m.grid && inr_shape_supported(m); }

int32_t train_n_weights(const InrDev& m) { return m.hidden * m.in + m.hidden * m.hidden + m.hidden; }

// Weight gradients (written), table gradient (accumulated into g_table) and
// mean loss of n points; `partial` holds max_waves * (NW + 1) floats.
hipError_t train_gradients(const InrDev& m, int prec, const float* u, const float* target, int64_t n, float scale,
                           float* g_table, float* g_weights, float* loss, float* partial, int64_t max_waves,
                           hipStream_t s) {
    TrainArgs a{u, target, n, scale, g_table, partial, 0, 0};
    int64_t used = 0;
    hipError_t e;
    const int NL = m.n_levels, F = m.n_features, H = m.hidden;
    if (NL == 8 && F == 2 && H == 32) e = launch_grad_p<8, 2, 32>(prec, m, a, max_waves, &used, s);
    else if (NL == 8 && F == 2 && H == 64) e = launch_grad_p<8, 2, 64>(prec, m, a, max_waves, &used, s);
    else if (NL == 16 && F == 2 && H == 32) e = launch_grad_p<16, 2, 32>(prec, m, a, max_waves, &used, s);
    else if (NL == 16 && F == 2 && H == 64) e = launch_grad_p<16, 2, 64>(prec, m, a, max_waves, &used, s);
    else if (NL == 16 && F == 4 && H == 64) e = launch_grad_p<16, 4, 64>(prec, m, a, max_waves, &used, s);
    else return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    const int32_t nw = train_n_weights(m);
    hipLaunchKernelGGL(k_train_reduce, dim3((nw + 1 + 255) / 256), dim3(256), 0, s, partial, used, nw, g_weights, loss,
                       n > 0 ? 1.0f / (float)n : 0.0f);
    return hipGetLastError();
}

hipError_t train_points(uint64_t seed, int64_t step, int64_t n, const float* grid, const int32_t dims[3], float* u,
                        float* target, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_train_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, step, n, grid,
                       dims ? dims[0] : 0, dims ? dims[1] : 0, dims ? dims[2] : 0, u, target);
    return hipGetLastError();
}

hipError_t adam_update(float* p, float* m1, float* m2, float* g, int64_t n, float lr, float b1, float b2, float eps,
                       int64_t step, bool clear, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const double c1 = 1.0 - pow((double)b1, (double)step), c2 = 1.0 - pow((double)b2, (double)step);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, p, m1, m2, g, n, lr, b1, b2, eps,
                       (float)(1.0 / c1), (float)(1.0 / c2), clear ? 1 : 0);
    return hipGetLastError();
}

hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace cinr
