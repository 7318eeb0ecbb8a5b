/*
 * cinr_oracle.c -- TEST INFRASTRUCTURE ONLY (see cinr_oracle.h).
 *
 * A plain CPU implementation of the paper's per-frame hot path, written for
 * readability: hash-grid encoding and MLP (Section 3), value normalisation
 * (Section 4.1), LoD lattice and bricks with one shared sample between
 * neighbours (Section 4.3.2), multi-resolution page-table lookup with
 * fallback to coarser LoDs (Section 4.3), priority ranking of requests
 * (Section 4.3.3), true-miss inference (Section 4.3.4, Algorithms 1 and 2),
 * stochastic LoD (Section 5.3), macro-cell empty-space skipping (Section 5.2)
 * and front-to-back ray marching (Section 5.1).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math (x86-64 SSE, so
 * every float expression below is one correctly rounded binary32 operation).
 */
#include "cinr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Threads                                                                    */
/* ------------------------------------------------------------------------- */

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Published generators                                                       */
/* ------------------------------------------------------------------------- */

/* SplitMix64 (Steele, Lea, Flood 2014): advance the state by the golden gamma,
 * then apply the variant-13 finaliser. */
uint64_t orc_splitmix64(uint64_t state) {
    uint64_t z = state + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Marsaglia (2003) xorshift on 32 bits with the shift triple (13, 17, 5). */
uint32_t orc_xorshift32(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

/* Per-frame seed of the stochastic LoD (Section 5.3: a light xorshift seeded
 * by a higher-quality value drawn once per frame): the high 32 bits of one
 * SplitMix64 output whose state is (seed << 32) | frame. */
uint32_t orc_frame_seed(uint32_t seed, uint32_t frame) {
    return (uint32_t)(orc_splitmix64(((uint64_t)seed << 32) | (uint64_t)frame) >> 32);
}

/* Philox-4x32 with 10 rounds (Salmon et al. 2011). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------- */
/* Hash-grid INR (Section 3)                                                  */
/* ------------------------------------------------------------------------- */

int64_t orc_level_size(const orc_inr* m, int level) {
    int64_t side = (int64_t)m->level_res[level] + 1;
    int64_t dense = side * side * side;
    int64_t T = (int64_t)1 << m->log2_table;
    return dense <= T ? dense : T;
}

int64_t orc_table_entries(const orc_inr* m) {
    int64_t s = 0;
    for (int l = 0; l < m->n_levels; ++l) s += orc_level_size(m, l);
    return s;
}

/* Table index of grid corner c at one level: the corner's dense index when the
 * whole (N+1)^3 grid fits in the table, otherwise the spatial hash of Mueller
 * et al. (2022), XOR of coordinate times (1, 2654435761, 805459861) in uint32
 * arithmetic, modulo the table size. */
static int64_t grid_index(int64_t cx, int64_t cy, int64_t cz, int64_t side, int dense, int64_t T) {
    if (dense) return cx + cy * side + cz * side * side;
    uint32_t h = ((uint32_t)cx * 1u) ^ ((uint32_t)cy * 2654435761u) ^ ((uint32_t)cz * 805459861u);
    return (int64_t)(h % (uint64_t)T);
}

/* Level l's feature vector at u in [0,1)^3: trilinear interpolation of the 8
 * surrounding grid points of the N_l grid; features concatenated level-major. */
static void encode_one(const orc_inr* m, const double u[3], double* feat) {
    const int F = m->n_features;
    const int64_t T = (int64_t)1 << m->log2_table;
    int64_t off = 0;
    for (int l = 0; l < m->n_levels; ++l) {
        const int64_t N = m->level_res[l];
        const int64_t side = N + 1;
        const int dense = side * side * side <= T;
        double w[3];
        int64_t c0[3];
        for (int a = 0; a < 3; ++a) {
            double s = u[a] * (double)N;
            double fl = floor(s);
            c0[a] = (int64_t)fl;
            w[a] = s - fl;
        }
        for (int j = 0; j < F; ++j) feat[l * F + j] = 0.0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
                    int64_t idx = grid_index(c0[0] + dx, c0[1] + dy, c0[2] + dz, side, dense, T);
                    const float* e = m->table + (off + idx) * F;
                    for (int j = 0; j < F; ++j) feat[l * F + j] += wt * (double)e[j];
                }
        off += orc_level_size(m, l);
    }
}

void orc_encode(const orc_inr* m, const double* u, int64_t n, double* feat) {
    const int nf = m->n_levels * m->n_features;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) encode_one(m, u + 3 * i, feat + nf * i);
}

/* Fully connected layers, no biases, ReLU between layers, linear output. */
static double mlp_one(const orc_inr* m, const double* feat) {
    double bufa[256], bufb[256];
    double* h = bufa;
    double* o = bufb;
    for (int i = 0; i < m->widths[0]; ++i) h[i] = feat[i];
    const float* W = m->weights;
    for (int k = 0; k < m->n_layers; ++k) {
        const int ni = m->widths[k], no = m->widths[k + 1];
        for (int r = 0; r < no; ++r) {
            double s = 0.0;
            for (int c = 0; c < ni; ++c) s += (double)W[r * ni + c] * h[c];
            o[r] = (k + 1 < m->n_layers && s < 0.0) ? 0.0 : s;
        }
        W += ni * no;
        double* t = h;
        h = o;
        o = t;
    }
    return h[0];
}

void orc_mlp(const orc_inr* m, const double* feat, int64_t n, double* y) {
    const int nf = m->widths[0];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = mlp_one(m, feat + nf * i);
}

/* Trilinear interpolation of the explicit grid at voxel coordinate x
 * (clamped to [0, V-1]; the last cell serves the upper faces). */
static double grid_value(const orc_inr* m, const double x[3]) {
    int64_t j[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double xa = x[a];
        const double hi = (double)(m->dims[a] - 1);
        if (xa < 0.0) xa = 0.0;
        if (xa > hi) xa = hi;
        int64_t ja = (int64_t)floor(xa);
        if (ja > m->dims[a] - 2) ja = m->dims[a] - 2;
        j[a] = ja;
        f[a] = xa - (double)ja;
    }
    const int64_t sy = m->dims[0], sz = (int64_t)m->dims[0] * m->dims[1];
    double v = 0.0;
    for (int k = 0; k < 8; ++k) {
        const int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
        const double w = (bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) * (bz ? f[2] : 1.0 - f[2]);
        v += w * (double)m->grid[(j[2] + bz) * sz + (j[1] + by) * sy + j[0] + bx];
    }
    return v;
}

/* Normalised INR value at LoD-0 voxel coordinate x: the coordinate is
 * clamped to [0, V-1], mapped to u = (x + 0.5) / V inside (0,1)^3, encoded,
 * passed through the MLP, then de-normalised with the stored value range and
 * clamped to [0,1] (Section 4.1: training runs on [0,1)^3 and [0,1] data).
 * An explicit-grid source replaces encoding and MLP by grid_value. */
static double value_one(const orc_inr* m, const double x[3]) {
    double u[3];
    double feat[ORC_MAX_LEVELS * 8];
    double y;
    if (m->grid) {
        y = grid_value(m, x);
    } else {
        for (int a = 0; a < 3; ++a) {
            double xa = x[a];
            double hi = (double)(m->dims[a] - 1);
            if (xa < 0.0) xa = 0.0;
            if (xa > hi) xa = hi;
            u[a] = (xa + 0.5) / (double)m->dims[a];
        }
        encode_one(m, u, feat);
        y = mlp_one(m, feat);
    }
    double v = (double)m->value_scale * y + (double)m->value_offset;
    if (v < 0.0) v = 0.0;
    if (v > 1.0) v = 1.0;
    return v;
}

void orc_value(const orc_inr* m, const double* x, int64_t n, double* v) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) v[i] = value_one(m, x + 3 * i);
}

/* ------------------------------------------------------------------------- */
/* LoD lattice and bricks (Section 4.3.2)                                     */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t K[3];  /* lattice points per axis at this LoD */
    int32_t nb[3]; /* bricks per axis */
    int64_t off;   /* first key of this LoD */
    int64_t count;
} lod_geom;

/* At LoD L the lattice spacing is 2^L voxels: K = ceil((V-1)/2^L) + 1 points
 * per axis.  Bricks hold B samples per axis and advance by B-1 samples, so
 * neighbours share one sample on each face (the paper's one-voxel covering). */
static void make_geom(const int32_t dims[3], int32_t B, int32_t L, int64_t off, lod_geom* g) {
    for (int a = 0; a < 3; ++a) {
        int64_t span = (int64_t)dims[a] - 1;
        int64_t step = (int64_t)1 << L;
        g->K[a] = (int32_t)((span + step - 1) / step + 1);
        g->nb[a] = (int32_t)(((int64_t)g->K[a] - 1 + (B - 1) - 1) / (B - 1));
    }
    g->off = off;
    g->count = (int64_t)g->nb[0] * g->nb[1] * g->nb[2];
}

int orc_lod_geometry(const int32_t dims[3], int32_t brick, int32_t n_lods, int32_t* K, int32_t* nb,
                     int64_t* key_offset) {
    if (brick < 2 || n_lods < 1 || n_lods > ORC_MAX_LODS) return -1;
    int64_t off = 0;
    for (int L = 0; L < n_lods; ++L) {
        lod_geom g;
        make_geom(dims, brick, L, off, &g);
        for (int a = 0; a < 3; ++a) {
            if (K) K[3 * L + a] = g.K[a];
            if (nb) nb[3 * L + a] = g.nb[a];
        }
        if (key_offset) key_offset[L] = off;
        off += g.count;
    }
    if (key_offset) key_offset[n_lods] = off;
    return 0;
}

/* The worked example of Section 4.3.2 taken literally: per axis the origin is
 * b * B * 2^L, minus one for every brick after the first.  Kept for the pin
 * only; bricks are generated with the shared-sample stride B-1 (see
 * decode_brick). */
void orc_brick_origin_literal(const int32_t b[3], int32_t lod, int32_t brick, int64_t out[3]) {
    for (int a = 0; a < 3; ++a) out[a] = (int64_t)b[a] * brick * ((int64_t)1 << lod) - (b[a] > 0 ? 1 : 0);
}

/* Brick (L, b): samples i in [0,B)^3 in (z, y, x) order at lattice index
 * b*(B-1) + i, i.e. at voxel coordinate clamp((b*(B-1) + i) * 2^L, 0, V-1). */
static void decode_brick(const orc_inr* m, int32_t L, const int32_t b[3], int32_t B, double* out) {
    for (int k = 0; k < B; ++k)
        for (int j = 0; j < B; ++j)
            for (int i = 0; i < B; ++i) {
                int64_t li[3] = {(int64_t)b[0] * (B - 1) + i, (int64_t)b[1] * (B - 1) + j,
                                 (int64_t)b[2] * (B - 1) + k};
                double x[3];
                for (int a = 0; a < 3; ++a) {
                    int64_t xa = li[a] << L;
                    if (xa > m->dims[a] - 1) xa = m->dims[a] - 1;
                    x[a] = (double)xa;
                }
                out[((int64_t)k * B + j) * B + i] = value_one(m, x);
            }
}

int orc_decode_bricks(const orc_inr* m, const int32_t* reqs, int64_t n, int32_t B, int32_t n_lods,
                      double* out) {
    int64_t off = 0;
    lod_geom g[ORC_MAX_LODS];
    if (B < 2 || n_lods < 1 || n_lods > ORC_MAX_LODS) return -1;
    for (int L = 0; L < n_lods; ++L) {
        make_geom(m->dims, B, L, off, &g[L]);
        off += g[L].count;
    }
    for (int64_t r = 0; r < n; ++r) {
        const int32_t* q = reqs + 4 * r;
        if (q[0] < 0 || q[0] >= n_lods) return -1;
        for (int a = 0; a < 3; ++a)
            if (q[1 + a] < 0 || q[1 + a] >= g[q[0]].nb[a]) return -1;
    }
    const int64_t B3 = (int64_t)B * B * B;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n; ++r) decode_brick(m, reqs[4 * r], reqs + 4 * r + 1, B, out + r * B3);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Macro-cells (Section 5.2)                                                  */
/* ------------------------------------------------------------------------- */

/* ceil(V/N) cells per axis; each stores min and max of the LoD-0 lattice
 * values inside its closed region [cN, min((c+1)N, V-1)]^3. */
void orc_macrocells(const orc_inr* m, int32_t N, float* minmax) {
    int32_t M[3];
    for (int a = 0; a < 3; ++a) M[a] = (m->dims[a] + N - 1) / N;
    const int64_t nc = (int64_t)M[0] * M[1] * M[2];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nc; ++c) {
        int32_t ci[3] = {(int32_t)(c % M[0]), (int32_t)((c / M[0]) % M[1]), (int32_t)(c / ((int64_t)M[0] * M[1]))};
        int32_t lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = ci[a] * N;
            hi[a] = (ci[a] + 1) * N;
            if (hi[a] > m->dims[a] - 1) hi[a] = m->dims[a] - 1;
        }
        double vmin = 1e300, vmax = -1e300;
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    double p[3] = {x, y, z};
                    double v = value_one(m, p);
                    if (v < vmin) vmin = v;
                    if (v > vmax) vmax = v;
                }
        minmax[2 * c] = (float)vmin;
        minmax[2 * c + 1] = (float)vmax;
    }
}

/* Maximum opacity over the transfer-function rows a cell's value range can
 * touch, [floor(min*255), ceil(max*255)]; the flag is 0 exactly when that
 * maximum is 0 (fully transparent cell, skipped by the sampler). */
/* Maximum opacity over the rows [floor(min*255), ceil(max*255)] of cell c. */
static float cell_mu(const float* minmax, int64_t c, const float* tf) {
    float a = minmax[2 * c] * 255.0f;
    float b = minmax[2 * c + 1] * 255.0f;
    int lo = (int)floorf(a), hi = (int)ceilf(b);
    if (lo < 0) lo = 0;
    if (hi > 255) hi = 255;
    float mu = 0.0f;
    for (int r = lo; r <= hi; ++r)
        if (tf[4 * r + 3] > mu) mu = tf[4 * r + 3];
    return mu;
}

/* floor(-log2 mu) for 0 < mu < 1 from the binary32 fields: mu = m 2^x with
 * m in [1, 2) gives -log2 mu in (-x - 1, -x], equal to -x exactly when m = 1. */
int32_t orc_step_exp(float mu, int32_t E) {
    if (mu >= 1.0f) return 0;
    uint32_t bits;
    memcpy(&bits, &mu, 4);
    const int32_t x = (int32_t)((bits >> 23) & 0xFFu) - 127;
    const int32_t e = (bits & 0x7FFFFFu) == 0u ? -x : -x - 1;
    return e < E ? e : E;
}

void orc_macrocell_step_codes(const float* minmax, int64_t n_cells, const float* tf, int32_t E, uint8_t* codes) {
    for (int64_t c = 0; c < n_cells; ++c) {
        const float mu = cell_mu(minmax, c, tf);
        codes[c] = mu > 0.0f ? (uint8_t)orc_step_exp(mu, E) : (uint8_t)0xFF;
    }
}

void orc_macrocell_flags(const float* minmax, int64_t n_cells, const float* tf, uint8_t* flags) {
    for (int64_t c = 0; c < n_cells; ++c) {
        float a = minmax[2 * c] * 255.0f;
        float b = minmax[2 * c + 1] * 255.0f;
        int lo = (int)floorf(a), hi = (int)ceilf(b);
        if (lo < 0) lo = 0;
        if (hi > 255) hi = 255;
        float mu = 0.0f;
        for (int r = lo; r <= hi; ++r)
            if (tf[4 * r + 3] > mu) mu = tf[4 * r + 3];
        flags[c] = mu > 0.0f ? 1 : 0;
    }
}

/* ------------------------------------------------------------------------- */
/* Decision plane (binary32)                                                  */
/* ------------------------------------------------------------------------- */

/* Primary ray through the centre of pixel (i, j), row 0 at the top, and its
 * parametric overlap [ts, te] with the box [0, V-1]^3 (slab test).  Returns 0
 * when the ray misses the box. */
int orc_ray_setup(const orc_camera* c, const int32_t dims[3], int32_t i, int32_t j, float o[3], float d[3],
                  float* ts, float* te) {
    float fx = ((float)i + 0.5f) / (float)c->width;
    float fy = ((float)j + 0.5f) / (float)c->height;
    if (c->projection == 0) {
        float sx = (fx * 2.0f - 1.0f) * c->tan_half_x;
        float sy = (1.0f - fy * 2.0f) * c->tan_half_y;
        float dir[3];
        for (int a = 0; a < 3; ++a) {
            float r = sx * c->right[a];
            float s = c->forward[a] + r;
            float u = sy * c->up[a];
            dir[a] = s + u;
        }
        float n2 = dir[0] * dir[0];
        float y2 = dir[1] * dir[1];
        float z2 = dir[2] * dir[2];
        n2 = n2 + y2;
        n2 = n2 + z2;
        float n = sqrtf(n2);
        for (int a = 0; a < 3; ++a) {
            d[a] = dir[a] / n;
            o[a] = c->eye[a];
        }
    } else {
        float ox = (fx - 0.5f) * c->ortho_w;
        float oy = (0.5f - fy) * c->ortho_h;
        for (int a = 0; a < 3; ++a) {
            float r = ox * c->right[a];
            float s = c->eye[a] + r;
            float u = oy * c->up[a];
            o[a] = s + u;
            d[a] = c->forward[a];
        }
    }
    float tlo = -INFINITY, thi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        float hi = (float)(dims[a] - 1);
        if (d[a] == 0.0f) {
            if (o[a] < 0.0f || o[a] > hi) return 0;
            continue;
        }
        float ta = (0.0f - o[a]) / d[a];
        float tb = (hi - o[a]) / d[a];
        float lo_ = ta < tb ? ta : tb;
        float hi_ = ta < tb ? tb : ta;
        if (lo_ > tlo) tlo = lo_;
        if (hi_ < thi) thi = hi_;
    }
    float t0 = tlo > 0.0f ? tlo : 0.0f;
    if (!(thi >= t0) || !(thi < INFINITY)) return 0; /* degenerate direction: no samples */
    *ts = t0;
    *te = thi;
    return 1;
}

static uint32_t float_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Algorithm 2 with Section 5.3: D = |p - eye| * lod_scale; the LoD is the
 * integer part of D, moved one level coarser when a uniform variate drawn by
 * xorshift from (bits of D) XOR (frame seed) falls below the fractional part,
 * so that the expected LoD equals D.  Then clamped to [lod_floor, n_lods-1]. */
int32_t orc_select_lod(const float p[3], const float eye[3], float lod_scale, uint32_t frame_seed,
                       int32_t lod_floor, int32_t n_lods) {
    return orc_select_lod_scaled(p, eye, lod_scale, 1.0f, frame_seed, lod_floor, n_lods);
}

/* The same with the distance scaled by `factor` (context-aware LoD):
 * D = (|p - eye| * lod_scale) * factor. */
int32_t orc_select_lod_scaled(const float p[3], const float eye[3], float lod_scale, float factor,
                              uint32_t frame_seed, int32_t lod_floor, int32_t n_lods) {
    float dx = p[0] - eye[0];
    float dy = p[1] - eye[1];
    float dz = p[2] - eye[2];
    float s = dx * dx;
    float sy = dy * dy;
    float sz = dz * dz;
    s = s + sy;
    s = s + sz;
    float D0 = sqrtf(s) * lod_scale;
    float D = D0 * factor;
    float fl = floorf(D);
    float fr = D - fl;
    uint32_t r = orc_xorshift32(float_bits(D) ^ frame_seed);
    float u = (float)(r >> 8) * 5.9604644775390625e-08f; /* 2^-24 */
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

/* Section 4.3.4 pre-load: start with every sample at the coarsest LoD, then
 * release one LoD every `period` frames. */
int32_t orc_lod_floor(int32_t frame, int32_t period, int32_t n_lods) {
    if (period <= 0) return 0;
    int32_t f = n_lods - 1 - frame / period;
    return f < 0 ? 0 : f;
}

/* Section 4.3.4 pre-load, continued: the frames whose samples are all forced
 * to the coarsest LoD (the first `period` frames) march every ray to the end
 * of the volume, with early ray termination suspended, so that the coarsest
 * bricks behind opaque material are requested too and the cache holds a
 * low-resolution copy of nearly the whole volume to fall back on. */
int32_t orc_preload_frame(int32_t frame, int32_t period) { return period > 0 && frame >= 0 && frame < period; }

/* ------------------------------------------------------------------------- */
/* Value plane helpers                                                        */
/* ------------------------------------------------------------------------- */

/* Transfer function (Section 3): linear interpolation between rows
 * floor(v*255) and the next one. */
static void tf_lookup(const float* tf, double v, double rgba[4]) {
    double x = v * 255.0;
    int i0 = (int)floor(x);
    if (i0 > 254) i0 = 254;
    if (i0 < 0) i0 = 0;
    double t = x - (double)i0;
    for (int c = 0; c < 4; ++c) rgba[c] = (double)tf[4 * i0 + c] * (1.0 - t) + (double)tf[4 * (i0 + 1) + c] * t;
}

typedef struct {
    double C[3], A;
} ray_acc;

/* Front-to-back compositing with opacity corrected from a one-voxel
 * reference length to the step: a' = 1 - (1 - a)^step. */
static void composite(ray_acc* acc, const float* tf, double v, double step) {
    double rgba[4];
    tf_lookup(tf, v, rgba);
    double a = rgba[3];
    if (a > 1.0) a = 1.0;
    if (a < 0.0) a = 0.0;
    double ac = 1.0 - pow(1.0 - a, step);
    double wgt = (1.0 - acc->A) * ac;
    for (int c = 0; c < 3; ++c) acc->C[c] += wgt * rgba[c];
    acc->A += wgt;
}

static double trilinear8(const double c[8], const double f[3]) {
    double x00 = c[0] * (1.0 - f[0]) + c[1] * f[0];
    double x10 = c[2] * (1.0 - f[0]) + c[3] * f[0];
    double x01 = c[4] * (1.0 - f[0]) + c[5] * f[0];
    double x11 = c[6] * (1.0 - f[0]) + c[7] * f[0];
    double y0 = x00 * (1.0 - f[1]) + x10 * f[1];
    double y1 = x01 * (1.0 - f[1]) + x11 * f[1];
    return y0 * (1.0 - f[2]) + y1 * f[2];
}

/* ------------------------------------------------------------------------- */
/* Cache state (Section 4.3.1)                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t pix, k;
    float x, y, z;
} miss_rec;

struct orc_cache {
    orc_inr inr;                    /* volume 0 */
    orc_inr inrs[ORC_MAX_VOLS];     /* all volumes sharing the cache */
    int32_t n_vols;
    int64_t keys_per_vol;           /* volume v owns keys [v K, (v+1) K) */
    orc_cache_desc d;
    lod_geom g[ORC_MAX_LODS];
    int64_t n_keys;
    int32_t* pt;        /* key -> slot, -1 unmapped */
    int32_t* owner;     /* slot -> key, -1 free */
    int32_t* last_used; /* slot -> last frame that read it, -1 never */
    int64_t* rank;      /* key -> rank, -1 undefined */
    uint32_t* req;      /* key -> requests in the current frame */
    uint32_t* last_req; /* counts seen by the last end-of-frame step */
    double* pool;       /* slot -> B^3 values */
    int32_t* req_list;
    int64_t n_req_list;
    miss_rec* misses;
    int64_t n_misses;
    int log_misses;
    int32_t* evlog;
    int64_t n_evlog, cap_evlog;
    int trace_ert;
    int32_t* ert_trace; /* per pixel: samples whose decisions were made */
    int64_t n_ert_trace;
};

orc_cache* orc_cache_create(const orc_inr* m, const orc_cache_desc* d) { return orc_cache_create_multi(m, 1, d); }

orc_cache* orc_cache_create_multi(const orc_inr* ms, int32_t n_vols, const orc_cache_desc* d) {
    if (d->brick < 2 || d->n_lods < 1 || d->n_lods > ORC_MAX_LODS || d->pool_bricks < 0 || d->max_requests < 0)
        return NULL;
    if (n_vols < 1 || n_vols > ORC_MAX_VOLS) return NULL;
    if (d->f16_lods) {
        const uint32_t all = d->n_lods >= 32 ? 0xFFFFFFFFu : (1u << d->n_lods) - 1u;
        const int32_t p16 = d->pool_bricks_f16, p32 = d->pool_bricks - d->pool_bricks_f16;
        if (d->pool_f16 || (d->f16_lods & ~all) || d->f16_lods == all || p16 < 1 || p32 < 1 ||
            d->max_requests > p16 || d->max_requests > p32)
            return NULL;
    }
    for (int i = 1; i < n_vols; ++i)
        for (int a = 0; a < 3; ++a)
            if (ms[i].dims[a] != ms[0].dims[a]) return NULL;
    orc_cache* c = (orc_cache*)calloc(1, sizeof(orc_cache));
    c->inr = ms[0];
    for (int i = 0; i < n_vols; ++i) c->inrs[i] = ms[i];
    c->n_vols = n_vols;
    c->d = *d;
    int64_t kpv = 0;
    for (int L = 0; L < d->n_lods; ++L) {
        make_geom(ms[0].dims, d->brick, L, kpv, &c->g[L]);
        kpv += c->g[L].count;
    }
    c->keys_per_vol = kpv;
    const int64_t off = kpv * n_vols;
    c->n_keys = off;
    const int64_t B3 = (int64_t)d->brick * d->brick * d->brick;
    c->pt = (int32_t*)malloc(sizeof(int32_t) * off);
    c->rank = (int64_t*)malloc(sizeof(int64_t) * off);
    c->req = (uint32_t*)calloc(off, sizeof(uint32_t));
    c->last_req = (uint32_t*)calloc(off, sizeof(uint32_t));
    const int64_t P = d->pool_bricks > 0 ? d->pool_bricks : 1;
    c->owner = (int32_t*)malloc(sizeof(int32_t) * P);
    c->last_used = (int32_t*)malloc(sizeof(int32_t) * P);
    if (!c->pt || !c->rank || !c->req || !c->last_req || !c->owner || !c->last_used) {
        orc_cache_destroy(c);
        return NULL;
    }
    for (int64_t k = 0; k < off; ++k) {
        c->pt[k] = -1;
        c->rank[k] = -1;
    }
    for (int64_t s = 0; s < P; ++s) {
        c->owner[s] = -1;
        c->last_used[s] = -1;
    }
    c->pool = (double*)calloc((size_t)(P * B3), sizeof(double));
    c->req_list = (int32_t*)malloc(sizeof(int32_t) * (d->max_requests > 0 ? d->max_requests : 1));
    c->cap_evlog = 1024;
    c->evlog = (int32_t*)malloc(sizeof(int32_t) * 4 * c->cap_evlog);
    if (!c->pool || !c->req_list || !c->evlog) {  // e.g. an FP64 pool larger than host memory
        orc_cache_destroy(c);
        return NULL;
    }
    return c;
}

void orc_cache_destroy(orc_cache* c) {
    if (!c) return;
    free(c->pt);
    free(c->rank);
    free(c->req);
    free(c->last_req);
    free(c->owner);
    free(c->last_used);
    free(c->pool);
    free(c->req_list);
    free(c->misses);
    free(c->evlog);
    free(c->ert_trace);
    free(c);
}

int64_t orc_cache_n_keys(const orc_cache* c) { return c->n_keys; }
void orc_cache_page_table(const orc_cache* c, int32_t* out) { memcpy(out, c->pt, sizeof(int32_t) * c->n_keys); }
void orc_cache_owner(const orc_cache* c, int32_t* out) { memcpy(out, c->owner, sizeof(int32_t) * c->d.pool_bricks); }
void orc_cache_last_used(const orc_cache* c, int32_t* out) {
    memcpy(out, c->last_used, sizeof(int32_t) * c->d.pool_bricks);
}
void orc_cache_rank(const orc_cache* c, int64_t* out) { memcpy(out, c->rank, sizeof(int64_t) * c->n_keys); }
void orc_cache_req_count(const orc_cache* c, uint32_t* out) {
    memcpy(out, c->last_req, sizeof(uint32_t) * c->n_keys);
}
int64_t orc_cache_request_list(const orc_cache* c, int32_t* out) {
    if (out) memcpy(out, c->req_list, sizeof(int32_t) * c->n_req_list);
    return c->n_req_list;
}
int64_t orc_cache_miss_list(const orc_cache* c, int32_t* pix_k, float* pos, int64_t cap) {
    int64_t n = c->n_misses < cap ? c->n_misses : cap;
    for (int64_t i = 0; i < n; ++i) {
        pix_k[2 * i] = c->misses[i].pix;
        pix_k[2 * i + 1] = c->misses[i].k;
        pos[3 * i] = c->misses[i].x;
        pos[3 * i + 1] = c->misses[i].y;
        pos[3 * i + 2] = c->misses[i].z;
    }
    return c->n_misses;
}
int64_t orc_cache_evict_log(const orc_cache* c, int32_t* out, int64_t cap) {
    int64_t n = c->n_evlog < cap ? c->n_evlog : cap;
    if (out) memcpy(out, c->evlog, sizeof(int32_t) * 4 * n);
    return c->n_evlog;
}
void orc_cache_pool(const orc_cache* c, double* out) {
    const int64_t B3 = (int64_t)c->d.brick * c->d.brick * c->d.brick;
    memcpy(out, c->pool, sizeof(double) * B3 * c->d.pool_bricks);
}
void orc_cache_set_miss_logging(orc_cache* c, int on) { c->log_misses = on; }
void orc_cache_set_ert_trace(orc_cache* c, int on) { c->trace_ert = on; }
int64_t orc_cache_ert_trace(const orc_cache* c, int32_t* out, int64_t cap) {
    int64_t n = c->n_ert_trace < cap ? c->n_ert_trace : cap;
    if (out && c->ert_trace) memcpy(out, c->ert_trace, sizeof(int32_t) * n);
    return c->n_ert_trace;
}

/* LoD of a key (of any volume sharing the cache). */
static int key_lod(const orc_cache* c, int64_t key) {
    const int64_t k = key % c->keys_per_vol;
    int L = 0;
    while (L + 1 < c->d.n_lods && k >= c->g[L + 1].off) ++L;
    return L;
}

/* First binary16 slot: the pool's binary16 class is [split, pool_bricks);
 * pool_bricks when the pool has one class. */
static int32_t f16_split(const orc_cache* c) {
    return c->d.f16_lods ? c->d.pool_bricks - c->d.pool_bricks_f16 : c->d.pool_bricks;
}

/* Slots [lo, hi) of the class a key's bricks are stored in. */
static void key_slots(const orc_cache* c, int64_t key, int32_t* lo, int32_t* hi) {
    const int32_t split = f16_split(c);
    if (c->d.f16_lods && ((c->d.f16_lods >> key_lod(c, key)) & 1u)) {
        *lo = split;
        *hi = c->d.pool_bricks;
    } else {
        *lo = 0;
        *hi = split;
    }
}

/* Insert one brick (Figure 1 step (5)): lowest free slot, otherwise the least
 * recently used slot by (last_used, slot) among slots not filled by this
 * batch, both among the slots of the brick's class (the whole pool unless
 * the pool mixes binary32 and binary16 LoDs).  The evicted brick's
 * page-table entry is unmapped and its rank forgotten; the new brick is
 * decoded into the slot, mapped, and stamped. */
static void insert_brick(orc_cache* c, int32_t key, int32_t stamp, uint8_t* filled, int32_t* slot_out) {
    int32_t lo, hi;
    key_slots(c, key, &lo, &hi);
    int32_t slot = -1;
    for (int32_t s = lo; s < hi; ++s)
        if (c->owner[s] < 0) {
            slot = s;
            break;
        }
    if (slot < 0) {
        for (int32_t s = lo; s < hi; ++s) {
            if (filled[s]) continue;
            if (slot < 0 || c->last_used[s] < c->last_used[slot]) slot = s;
        }
    }
    *slot_out = -1;
    if (slot < 0) return;
    int32_t old = c->owner[slot];
    if (old >= 0) {
        c->pt[old] = -1;
        c->rank[old] = -1;
    }
    *slot_out = slot;
    c->pt[key] = slot;
    c->owner[slot] = key;
    c->last_used[slot] = stamp;
    filled[slot] = 1;
    if (c->n_evlog == c->cap_evlog) {
        c->cap_evlog *= 2;
        c->evlog = (int32_t*)realloc(c->evlog, sizeof(int32_t) * 4 * c->cap_evlog);
    }
    int32_t* e = c->evlog + 4 * c->n_evlog++;
    e[0] = stamp;
    e[1] = slot;
    e[2] = old;
    e[3] = key;
}

double orc_round_half(double x) {
    if (x == 0.0 || isnan(x) || isinf(x)) return x;
    const double a = fabs(x);
    int e2;
    frexp(a, &e2);                       /* a = f 2^e2, f in [0.5, 1): the leading bit has weight 2^(e2-1) */
    int lead = e2 - 1;
    if (lead < -14) lead = -14;          /* below the normal range the spacing stays 2^-24 */
    const double quantum = ldexp(1.0, lead - 10);
    double q = a / quantum;              /* exact: a division by a power of two */
    const double fl = floor(q), rem = q - fl;
    q = rem > 0.5 ? fl + 1.0 : rem < 0.5 ? fl : (fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0);
    const double r = q * quantum;
    if (r > 65504.0) return x > 0 ? INFINITY : -INFINITY;
    return x > 0 ? r : -r;
}

/* Decodes the bricks just inserted (key -> slot) into their pool slots. */
static void decode_inserted(orc_cache* c, const int32_t* keys, const int32_t* slots, int64_t n) {
    const int64_t B3 = (int64_t)c->d.brick * c->d.brick * c->d.brick;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        if (slots[i] < 0) continue;
        const int32_t vol = (int32_t)(keys[i] / c->keys_per_vol);
        const int64_t key = keys[i] - (int64_t)vol * c->keys_per_vol;
        int L = 0;
        while (L + 1 < c->d.n_lods && key >= c->g[L + 1].off) ++L;
        const int64_t local = key - c->g[L].off;
        const int32_t b[3] = {(int32_t)(local % c->g[L].nb[0]), (int32_t)((local / c->g[L].nb[0]) % c->g[L].nb[1]),
                              (int32_t)(local / ((int64_t)c->g[L].nb[0] * c->g[L].nb[1]))};
        double* dst = c->pool + (int64_t)slots[i] * B3;
        decode_brick(&c->inrs[vol], L, b, c->d.brick, dst);
        if (c->d.pool_f16 || slots[i] >= f16_split(c))
            for (int64_t v = 0; v < B3; ++v) dst[v] = orc_round_half(dst[v]);
    }
}

/* Pre-loading into free slots only (never evicts). */
int orc_cache_prefill(orc_cache* c, const int32_t* keys, int64_t n, int32_t stamp) {
    for (int64_t i = 0; i < n; ++i)
        if (keys[i] < 0 || keys[i] >= c->n_keys || c->pt[keys[i]] >= 0) return -1;
    /* every key needs a free slot of its class */
    const int32_t split = f16_split(c);
    int64_t n_free[2] = {0, 0}, need[2] = {0, 0};
    for (int32_t s = 0; s < c->d.pool_bricks; ++s) n_free[s >= split] += c->owner[s] < 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t lo, hi;
        key_slots(c, keys[i], &lo, &hi);
        need[lo > 0] += 1;  /* the binary16 class starts above slot 0 */
    }
    if (need[0] > n_free[0] || need[1] > n_free[1]) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            if (keys[i] == keys[j]) return -1;
    uint8_t* filled = (uint8_t*)calloc(c->d.pool_bricks > 0 ? c->d.pool_bricks : 1, 1);
    int32_t* slots = (int32_t*)malloc(sizeof(int32_t) * (n ? n : 1));
    for (int64_t i = 0; i < n; ++i) insert_brick(c, keys[i], stamp, filled, &slots[i]);
    decode_inserted(c, keys, slots, n);
    free(slots);
    free(filled);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sampler (Algorithm 2 with the fallback of Section 4.3)                     */
/* ------------------------------------------------------------------------- */

enum { S_HIT = 0, S_FALLBACK = 1, S_MISS = 2, S_SKIP = 3 };

typedef struct {
    const orc_inr* m;
    orc_cache* c;           /* NULL in the uncached modes */
    int64_t key_base;       /* first key of the frame's volume in a shared cache */
    int readonly;           /* no request counts, no stamps */
    const orc_camera* cam;
    const orc_params* p;
    const uint8_t* flags;   /* macro-cell flags or NULL */
    int32_t M[3];
    uint32_t frame_seed;
    int32_t lod_floor;
    int32_t preload;        /* a pre-load frame: early ray termination suspended */
    float vm1[3];
} frame_ctx;

typedef struct {
    int status;
    double value;
    float value32; /* the value in binary32, for decisions that depend on it (path tracing) */
    float pos[3];
    int exp;  /* step exponent of the sample's cell (0 without adaptive sampling) */
} sample_out;

/* Binary32 linear interpolation a + t (b - a), rounded once. */
static float lerp32(float a, float b, float t) { return fmaf(t, b - a, a); }

/* Trilinear interpolation in binary32, along x, then y, then z; corners
 * c[dx + 2 dy + 4 dz]. */
static float trilinear32(const float c[8], const float f[3]) {
    const float x00 = lerp32(c[0], c[1], f[0]), x10 = lerp32(c[2], c[3], f[0]);
    const float x01 = lerp32(c[4], c[5], f[0]), x11 = lerp32(c[6], c[7], f[0]);
    const float y0 = lerp32(x00, x10, f[1]), y1 = lerp32(x01, x11, f[1]);
    return lerp32(y0, y1, f[2]);
}

/* Binary32 value of a true miss: an explicit grid is interpolated in binary32
 * at the (clamped) position, then mapped by value_scale * v + value_offset
 * (rounded once) and clamped to [0, 1]; an INR's value is its FP64 value
 * rounded to binary32. */
static float miss_value32(const orc_inr* m, const float pos[3], double v64) {
    if (!m->grid) return (float)v64;
    float c[8], f[3];
    int32_t j[3];
    for (int a = 0; a < 3; ++a) {
        const float hi = (float)(m->dims[a] - 1);
        float xa = pos[a];
        if (xa < 0.0f) xa = 0.0f;
        if (xa > hi) xa = hi;
        j[a] = (int32_t)xa;
        if (j[a] > m->dims[a] - 2) j[a] = m->dims[a] - 2;
        f[a] = xa - (float)j[a];
    }
    const int64_t sy = m->dims[0], sz = (int64_t)m->dims[0] * m->dims[1];
    for (int n = 0; n < 8; ++n)
        c[n] = m->grid[(j[2] + ((n >> 2) & 1)) * sz + (j[1] + ((n >> 1) & 1)) * sy + j[0] + (n & 1)];
    float v = fmaf(m->value_scale, trilinear32(c, f), m->value_offset);
    if (v < 0.0f) v = 0.0f;
    if (v > 1.0f) v = 1.0f;
    return v;
}

typedef struct {
    int64_t samples, hits, fallbacks, misses, skipped, ert_violations;
    miss_rec* misses_buf;
    int64_t n_m, cap_m;
} thread_acc;

/* One sample of the sampler: position, macro-cell test, LoD, page-table
 * lookup at that LoD then at every coarser one; on a hit or fallback the
 * value is the trilinear interpolation of the serving brick and the slot is
 * stamped with the frame; otherwise the sample is a true miss.  Any sample
 * not served at its own LoD raises a request for its brick at that LoD. */
static void sample_decide(const frame_ctx* fc, const float o[3], const float d[3], float t, sample_out* so) {
    const orc_params* P = fc->p;
    so->exp = 0;
    so->value32 = 0.0f;
    float pos[3];
    for (int a = 0; a < 3; ++a) {
        float td = t * d[a];
        float q = o[a] + td;
        if (q < 0.0f) q = 0.0f;
        if (q > fc->vm1[a]) q = fc->vm1[a];
        pos[a] = q;
        so->pos[a] = q;
    }
    float lod_factor = 1.0f;
    if (fc->flags) {
        int32_t ci[3];
        for (int a = 0; a < 3; ++a) {
            ci[a] = (int32_t)pos[a] / P->macro_cell;
            if (ci[a] > fc->M[a] - 1) ci[a] = fc->M[a] - 1;
        }
        const int64_t cell = ((int64_t)ci[2] * fc->M[1] + ci[1]) * fc->M[0] + ci[0];
        const uint8_t code = fc->flags[cell];
        if (P->lod_context > 0.0f) {
            /* context-aware LoD: 1 - kappa * (value range of the cell), binary32 */
            const float range = P->macro_minmax[2 * cell + 1] - P->macro_minmax[2 * cell];
            const float k = P->lod_context * range;
            lod_factor = 1.0f - k;
        }
        if (P->adapt_max_exp >= 0) {
            /* adaptive rate: the cell's step exponent, the largest one across a transparent cell */
            if (code == 0xFF) {
                so->exp = P->adapt_max_exp;
                so->status = S_SKIP;
                so->value = 0.0;
                return;
            }
            so->exp = code;
        } else if (!code) {
            so->status = S_SKIP;
            so->value = 0.0;
            return;
        }
    }
    if (P->mode == ORC_UNCACHED_DIRECT) {
        so->status = S_MISS;
        return;
    }
    if (P->mode == ORC_UNCACHED_LATTICE) {
        double corner[8], f[3];
        int64_t j[3];
        for (int a = 0; a < 3; ++a) {
            j[a] = (int64_t)pos[a];
            if (j[a] > fc->m->dims[a] - 2) j[a] = fc->m->dims[a] - 2;
            f[a] = (double)(pos[a] - (float)j[a]);
        }
        float c32[8], f32[3];
        for (int n = 0; n < 8; ++n) {
            double x[3] = {(double)(j[0] + (n & 1)), (double)(j[1] + ((n >> 1) & 1)), (double)(j[2] + ((n >> 2) & 1))};
            corner[n] = value_one(fc->m, x);
            c32[n] = (float)corner[n];
        }
        for (int a = 0; a < 3; ++a) f32[a] = pos[a] - (float)j[a];
        so->status = S_HIT;
        so->value = trilinear8(corner, f);
        so->value32 = trilinear32(c32, f32);
        return;
    }
    orc_cache* c = fc->c;
    const int32_t B = c->d.brick;
    const int32_t nl = c->d.n_lods;
    const int32_t L = orc_select_lod_scaled(pos, fc->cam->eye, P->lod_scale, lod_factor, fc->frame_seed,
                                            fc->lod_floor, nl);
    int64_t req_key = -1;
    so->status = S_MISS;
    for (int32_t Lp = L; Lp < nl; ++Lp) {
        const lod_geom* g = &c->g[Lp];
        const float sc = ldexpf(1.0f, -Lp);
        float q[3];
        int32_t j[3], b[3];
        for (int a = 0; a < 3; ++a) {
            q[a] = pos[a] * sc;
            j[a] = (int32_t)q[a];
            if (j[a] > g->K[a] - 2) j[a] = g->K[a] - 2;
            b[a] = j[a] / (B - 1);
        }
        const int64_t key = g->off + ((int64_t)b[2] * g->nb[1] + b[1]) * g->nb[0] + b[0];
        if (Lp == L) req_key = key;
        const int32_t slot = c->pt[fc->key_base + key];
        if (slot < 0) continue;
        /* served by this brick */
        const int64_t B3 = (int64_t)B * B * B;
        const double* br = c->pool + (int64_t)slot * B3;
        int32_t l[3];
        double f[3], corner[8];
        float c32[8], f32[3];
        for (int a = 0; a < 3; ++a) {
            l[a] = j[a] - b[a] * (B - 1);
            f32[a] = q[a] - (float)j[a];
            f[a] = (double)f32[a];
        }
        for (int n = 0; n < 8; ++n) {
            int dx = n & 1, dy = (n >> 1) & 1, dz = (n >> 2) & 1;
            corner[n] = br[((int64_t)(l[2] + dz) * B + (l[1] + dy)) * B + (l[0] + dx)];
            c32[n] = (float)corner[n];
        }
        so->value = trilinear8(corner, f);
        so->value32 = trilinear32(c32, f32);
        so->status = (Lp == L) ? S_HIT : S_FALLBACK;
        if (!fc->readonly) {
#pragma omp atomic write
            c->last_used[slot] = P->frame_index;
        }
        break;
    }
    if (so->status != S_HIT && !fc->readonly) {
#pragma omp atomic
        c->req[fc->key_base + req_key] += 1u;
    }
}

static void acc_miss(thread_acc* ta, int32_t pix, int32_t k, const float pos[3]) {
    if (ta->n_m == ta->cap_m) {
        ta->cap_m = ta->cap_m ? ta->cap_m * 2 : 1024;
        ta->misses_buf = (miss_rec*)realloc(ta->misses_buf, sizeof(miss_rec) * ta->cap_m);
    }
    miss_rec* r = ta->misses_buf + ta->n_m++;
    r->pix = pix;
    r->k = k;
    r->x = pos[0];
    r->y = pos[1];
    r->z = pos[2];
}

/* Decide sample k, count it, and produce its value: a true miss is inferred
 * directly from the INR at the sample position (Algorithm 1, InferINR and
 * InsertMisses, within the same sampling step). */
static int run_sample(const frame_ctx* fc, thread_acc* ta, int32_t pix, int32_t k, const float o[3],
                      const float d[3], float ts, double* value, int* exp, int log_miss) {
    const float kk = (float)k * fc->p->step;
    const float t = ts + kk;
    sample_out so;
    sample_decide(fc, o, d, t, &so);
    ta->samples++;
    switch (so.status) {
        case S_HIT: ta->hits++; break;
        case S_FALLBACK: ta->fallbacks++; break;
        case S_SKIP: ta->skipped++; break;
        default: {
            ta->misses++;
            double x[3] = {so.pos[0], so.pos[1], so.pos[2]};
            so.value = value_one(fc->m, x);
            if (log_miss) acc_miss(ta, pix, k, so.pos);
        }
    }
    *value = so.value;
    *exp = so.exp;
    return so.status;
}

/* Number of samples t_k = ts + k*step with t_k <= te. */
static int32_t sample_count(float ts, float te, float step) {
    int32_t k = 0;
    for (;;) {
        float kk = (float)k * step;
        float t = ts + kk;
        if (t > te) return k;
        ++k;
    }
}

/* March one primary ray.  Samples are processed one by one and composited as
 * they come until the first true miss; from a true miss on, the next
 * `samples_per_iter` samples (the miss included) are gathered as one
 * wavefront step, their misses inferred, and then composited in order.  Early
 * termination is tested after every composited sample.  Without early
 * termination this is plain front-to-back compositing of every sample. */
/* Early termination after a composited sample; `knext` is the grid index of
 * the ray's next sample.  Without a replay: A >= threshold.  With a replay:
 * exactly where the checked renderer ended the ray, and a replayed end that
 * the oracle's own opacity contradicts by more than the slack (the checked
 * renderer's allowed value error, 1e-4 unless given) is counted. */
static int ert_end(const orc_params* P, thread_acc* ta, int32_t pix, int32_t knext, double A, double thr) {
    if (!P->ert_replay) return A >= thr;
    const double slack = P->ert_slack > 0.0 ? P->ert_slack : 1e-4;
    const int end = P->ert_replay[pix] == knext;
    if (end ? A < thr - slack : A >= thr + slack) ta->ert_violations++;
    return end;
}

static int32_t march(const frame_ctx* fc, thread_acc* ta, const float* tf, int32_t i, int32_t j, double out[4],
                     int log_miss) {
    const int32_t W = fc->cam->width;
    const int32_t pix = j * W + i;
    float o[3], d[3], ts, te;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    const orc_params* P = fc->p;
    if (P->ert_record) P->ert_record[pix] = -1;
    if (!orc_ray_setup(fc->cam, fc->m->dims, i, j, o, d, &ts, &te)) return 0;
    const int32_t nk = sample_count(ts, te, P->step);
    const int ert = P->ert_threshold <= 1.0f && !fc->preload;
    const double thr = (double)P->ert_threshold;
    const double step = (double)P->step;
    const int32_t S = P->samples_per_iter > 0 ? P->samples_per_iter : 1;
    ray_acc acc = {{0.0, 0.0, 0.0}, 0.0};
    double* vals = (double*)malloc(sizeof(double) * S);
    int* stat = (int*)malloc(sizeof(int) * S);
    int* exps = (int*)malloc(sizeof(int) * S);
    /* k: index of the next sample on the ray's grid t_k = ts + k*step; a
     * sample whose cell has step exponent e is followed by sample k + 2^e,
     * and its opacity is corrected to its own step 2^e*step */
    int32_t k = 0;
    int done = 0;
    while (!done && k < nk) {
        /* one sample at a time until the first true miss */
        int st = S_HIT, e = 0;
        double v = 0.0;
        while (k < nk) {
            st = run_sample(fc, ta, pix, k, o, d, ts, &v, &e, log_miss);
            if (st == S_MISS) break;
            if (st != S_SKIP) composite(&acc, tf, v, ldexp(step, e));
            k += 1 << e;
            if (ert && ert_end(P, ta, pix, k, acc.A, thr)) {
                done = 1;
                if (P->ert_record) P->ert_record[pix] = k;
                break;
            }
        }
        if (done || k >= nk) break;
        /* a wavefront step of S samples starting at the miss */
        int32_t n = 0;
        vals[n] = v;
        exps[n] = e;
        stat[n++] = st;
        int32_t kn = k + (1 << e);
        while (n < S && kn < nk) {
            stat[n] = run_sample(fc, ta, pix, kn, o, d, ts, &vals[n], &exps[n], log_miss);
            kn += 1 << exps[n];
            ++n;
        }
        int32_t kq = k; /* grid index after the composited samples */
        for (int32_t s = 0; s < n; ++s) {
            if (stat[s] != S_SKIP) composite(&acc, tf, vals[s], ldexp(step, exps[s]));
            kq += 1 << exps[s];
            if (ert && ert_end(P, ta, pix, kq, acc.A, thr)) {
                done = 1;
                if (P->ert_record) P->ert_record[pix] = kq;
                break;
            }
        }
        k = kn;
    }
    free(vals);
    free(stat);
    free(exps);
    out[0] = acc.C[0];
    out[1] = acc.C[1];
    out[2] = acc.C[2];
    out[3] = acc.A;
    return k;
}

/* ------------------------------------------------------------------------- */
/* Path tracing (Section 5.1: a second wavefront pipeline with Woodcock delta */
/* tracking through the same sampler)                                          */
/* ------------------------------------------------------------------------- */

/* The medium: extinction sigma(x) = pt_density * alpha(v(x)) with alpha the TF
 * opacity, so pt_density is a majorant; scattering albedo = TF colour at v;
 * isotropic phase function; one directional light toward pt_light_dir whose
 * term pt_light already carries the phase factor; the environment pt_ambient
 * lights scattered rays that leave the box.  Per path: delta tracking along
 * the primary ray; at every real collision the throughput takes the albedo,
 * a shadow ray toward the light is tracked the same way (transmittance 0 or
 * 1) and adds throughput * pt_light when it leaves the box, then the path
 * scatters isotropically, up to pt_max_bounces collisions.  A pixel's colour
 * is the mean radiance of its pt_spp paths, its opacity the fraction of paths
 * whose primary ray collides, over the paths completed within the event
 * budget ORC_PT_MAX_EVENTS.
 *
 * Randomness: Philox-4x32-10 with key (pt_seed, frame index) and counter
 * (pixel, n, 0, 0), n the pixel's event count (one draw per tentative
 * collision and per direction trial), continued across its paths. */

float orc_pt_uniform(uint32_t r) { return (float)(r >> 8) * 5.9604644775390625e-08f; }

float orc_pt_free_flight(uint32_t r) {
    const double xi = ((double)(r >> 8) + 1.0) * 5.9604644775390625e-08; /* exact, in (0, 1] */
    return (float)(-log(xi));
}

void orc_pt_free_flights(const uint32_t* words, int64_t n, float* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_pt_free_flight(words[i]);
}

float orc_pt_segment_exit(const float p[3], const float d[3], const float vm1[3]) {
    float t = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) continue;
        const float wall = d[a] > 0.0f ? vm1[a] : 0.0f;
        const float ta = (wall - p[a]) / d[a];
        if (ta < t) t = ta;
    }
    if (!(t >= 0.0f) || t == INFINITY) t = 0.0f;
    return t;
}

float orc_tf_alpha32(const float* tf, float v) {
    const float x = v * 255.0f;
    int32_t i0 = (int32_t)x;
    if (i0 > 254) i0 = 254;
    if (i0 < 0) i0 = 0;
    const float t = x - (float)i0;
    float a = lerp32(tf[4 * i0 + 3], tf[4 * (i0 + 1) + 3], t);
    if (a < 0.0f) a = 0.0f;
    if (a > 1.0f) a = 1.0f;
    return a;
}

static void pt_draw(uint32_t pix, uint32_t n, const uint32_t key[2], uint32_t r[4]) {
    const uint32_t ctr[4] = {pix, n, 0u, 0u};
    orc_philox4x32_10(ctr, key, r);
}

/* Marsaglia (1972): (u1, u2) uniform in the square [-1, 1)^2 until
 * s = u1^2 + u2^2 lies in (0, 1); then (2 u1 sqrt(1-s), 2 u2 sqrt(1-s), 1-2s)
 * is uniform on the unit sphere. */
static int marsaglia(const uint32_t r[4], float d[3]) {
    const float u1 = 2.0f * orc_pt_uniform(r[0]) - 1.0f;
    const float u2 = 2.0f * orc_pt_uniform(r[1]) - 1.0f;
    const float a = u1 * u1, b = u2 * u2;
    const float s = a + b;
    if (s >= 1.0f || s == 0.0f) return 0;
    const float q = sqrtf(1.0f - s);
    d[0] = (2.0f * u1) * q;
    d[1] = (2.0f * u2) * q;
    d[2] = 1.0f - 2.0f * s;
    return 1;
}

uint32_t orc_pt_direction(uint32_t pix, uint32_t n0, const uint32_t key[2], float d[3]) {
    uint32_t n = n0, r[4];
    do pt_draw(pix, n++, key, r);
    while (!marsaglia(r, d));
    return n;
}

#define PT_GATHER_MAX 8

typedef struct {
    const frame_ctx* fc;
    thread_acc* ta;
    const float* tf;
    int32_t pix;
    uint32_t key[2];
    uint32_t n;      /* next event */
    int capped;      /* the event budget is spent */
    int log_miss;
    int gather;      /* tentative collisions looked up from a true miss on: min(samples_per_iter, 8) */
    float inv_sigma; /* 1 / pt_density in binary32 */
} pt_ctx;

/* Position o + t d, clamped to the box (as the ray marcher's samples). */
static void pt_pos(const frame_ctx* fc, const float o[3], const float d[3], float t, float p[3]) {
    for (int a = 0; a < 3; ++a) {
        float td = t * d[a];
        float q = o[a] + td;
        if (q < 0.0f) q = 0.0f;
        if (q > fc->vm1[a]) q = fc->vm1[a];
        p[a] = q;
    }
}

/* One sampler lookup of tentative collision `event` at t: counted, requests
 * and stamps as for any sample, a true miss inferred (and logged with k =
 * event). */
static void pt_lookup(pt_ctx* c, const float o[3], const float d[3], float t, uint32_t event, sample_out* so) {
    const frame_ctx* fc = c->fc;
    thread_acc* ta = c->ta;
    sample_decide(fc, o, d, t, so);
    ta->samples++;
    switch (so->status) {
        case S_HIT: ta->hits++; break;
        case S_FALLBACK: ta->fallbacks++; break;
        case S_SKIP: ta->skipped++; break;
        default: {
            ta->misses++;
            double x[3] = {so->pos[0], so->pos[1], so->pos[2]};
            so->value = value_one(fc->m, x);
            so->value32 = miss_value32(fc->m, so->pos, so->value);
            if (c->log_miss) acc_miss(ta, c->pix, (int32_t)event, so->pos);
        }
    }
}

/* Woodcock delta tracking along o + t d from t0 to te: tentative collisions
 * at free-flight steps -ln(xi) / pt_density; a tentative collision is real
 * when a second uniform falls below the TF opacity at the sampled value
 * (decided in binary32; a skipped sample has opacity 0).  Returns 1 at a real
 * collision (its position and FP64 value), 0 when the segment is left or the
 * event budget ends.  From a true miss on, the next tentative collisions of
 * the segment (up to `gather` with the miss, those before te) are looked up
 * at once, as the wavefront step of the ray marcher; their values then serve
 * those events, and lookups beyond a real collision are unused. */
static int pt_track(pt_ctx* c, const float o[3], const float d[3], float t0, float te, float pos[3], double* v64) {
    sample_out g[PT_GATHER_MAX];
    uint32_t g_first = 0, g_n = 0; /* gathered events [g_first, g_first + g_n) */
    float t = t0;
    for (;;) {
        if (c->n >= ORC_PT_MAX_EVENTS) {
            c->capped = 1;
            return 0;
        }
        const uint32_t e = c->n++;
        uint32_t r[4];
        pt_draw(c->pix, e, c->key, r);
        const float step = orc_pt_free_flight(r[0]) * c->inv_sigma;
        t = t + step;
        if (t > te) return 0;
        sample_out so;
        if (e >= g_first && e < g_first + g_n) {
            so = g[e - g_first];
        } else {
            pt_lookup(c, o, d, t, e, &so);
            if (so.status == S_MISS) {
                g[0] = so;
                g_first = e;
                g_n = 1;
                float tg = t;
                while ((int)g_n < c->gather) {
                    const uint32_t eg = e + g_n;
                    uint32_t rg[4];
                    pt_draw(c->pix, eg, c->key, rg);
                    const float sg = orc_pt_free_flight(rg[0]) * c->inv_sigma;
                    tg = tg + sg;
                    if (tg > te) break;
                    pt_lookup(c, o, d, tg, eg, &g[g_n]);
                    ++g_n;
                }
            }
        }
        const float alpha = so.status == S_SKIP ? 0.0f : orc_tf_alpha32(c->tf, so.value32);
        if (orc_pt_uniform(r[1]) < alpha) {
            for (int a = 0; a < 3; ++a) pos[a] = so.pos[a];
            *v64 = so.value;
            return 1;
        }
    }
}

/* All pt_spp paths of pixel (i, j). */
static void pt_pixel(const frame_ctx* fc, thread_acc* ta, const float* tf, int32_t i, int32_t j, double out[4],
                     int log_miss) {
    const orc_params* P = fc->p;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    float o0[3], d0[3], ts, te;
    if (!orc_ray_setup(fc->cam, fc->m->dims, i, j, o0, d0, &ts, &te)) return;
    pt_ctx c;
    memset(&c, 0, sizeof(c));
    c.fc = fc;
    c.ta = ta;
    c.tf = tf;
    c.pix = j * fc->cam->width + i;
    c.key[0] = P->pt_seed;
    c.key[1] = (uint32_t)P->frame_index;
    c.log_miss = log_miss;
    c.gather = P->samples_per_iter < PT_GATHER_MAX ? P->samples_per_iter : PT_GATHER_MAX;
    if (c.gather < 1) c.gather = 1;
    c.inv_sigma = 1.0f / P->pt_density;
    double sum[3] = {0.0, 0.0, 0.0};
    int64_t hits = 0, done = 0;
    for (int32_t path = 0; path < P->pt_spp && !c.capped; ++path) {
        double beta[3] = {1.0, 1.0, 1.0}, L[3] = {0.0, 0.0, 0.0};
        int hit = 0;
        float o[3], d[3], t0 = ts, t1 = te;
        memcpy(o, o0, sizeof o);
        memcpy(d, d0, sizeof d);
        for (int32_t bounce = 0;;) {
            float p[3];
            double v;
            if (!pt_track(&c, o, d, t0, t1, p, &v)) {
                if (!c.capped && bounce > 0)
                    for (int k = 0; k < 3; ++k) L[k] += beta[k] * (double)P->pt_ambient[k];
                break;
            }
            if (bounce == 0) hit = 1;
            double rgba[4];
            tf_lookup(tf, v, rgba);
            for (int k = 0; k < 3; ++k) beta[k] *= rgba[k];
            /* next-event estimate: a shadow ray toward the light */
            const float tl = orc_pt_segment_exit(p, P->pt_light_dir, fc->vm1);
            float ps[3];
            double vs;
            const int blocked = pt_track(&c, p, P->pt_light_dir, 0.0f, tl, ps, &vs);
            if (c.capped) break;
            if (!blocked)
                for (int k = 0; k < 3; ++k) L[k] += beta[k] * (double)P->pt_light[k];
            if (++bounce == P->pt_max_bounces) break;
            /* isotropic scattering */
            int ok = 0;
            while (!ok) {
                if (c.n >= ORC_PT_MAX_EVENTS) {
                    c.capped = 1;
                    break;
                }
                uint32_t r[4];
                pt_draw(c.pix, c.n++, c.key, r);
                ok = marsaglia(r, d);
            }
            if (!ok) break;
            memcpy(o, p, sizeof o);
            t0 = 0.0f;
            t1 = orc_pt_segment_exit(p, d, fc->vm1);
        }
        if (c.capped) break; /* a path cut by the event budget is dropped */
        for (int k = 0; k < 3; ++k) sum[k] += L[k];
        hits += hit;
        done += 1;
    }
    if (done == 0) return;
    const double J = (double)done;
    out[0] = sum[0] / J;
    out[1] = sum[1] / J;
    out[2] = sum[2] / J;
    out[3] = (double)hits / J;
}

/* One pixel of the frame's pipeline. */
static void render_pixel(const frame_ctx* fc, thread_acc* ta, const float* tf, int32_t i, int32_t j, double out[4],
                         int log_miss, int32_t* nproc) {
    if (fc->p->pipeline == 1) {
        pt_pixel(fc, ta, tf, i, j, out, log_miss);
        if (nproc) *nproc = 0;
    } else {
        const int32_t k = march(fc, ta, tf, i, j, out, log_miss);
        if (nproc) *nproc = k;
    }
}

/* Parameters a frame needs: the context-aware LoD weight in [0, 1], and
 * those of the path tracer. */
static int params_ok(const orc_params* p) {
    if (!(p->lod_context >= 0.0f && p->lod_context <= 1.0f)) return 0;
    if (p->pipeline == 0) return 1;
    if (p->pipeline != 1) return 0;
    if (!(p->pt_density > 0.0f) || !isfinite(p->pt_density)) return 0;
    if (p->pt_spp < 1 || p->pt_max_bounces < 1 || p->adapt_max_exp >= 0) return 0;
    return 1;
}

static int cmp_miss(const void* a, const void* b) {
    const miss_rec* x = (const miss_rec*)a;
    const miss_rec* y = (const miss_rec*)b;
    if (x->pix != y->pix) return x->pix < y->pix ? -1 : 1;
    return (x->k > y->k) - (x->k < y->k);
}

static int render_pass(frame_ctx* fc, const float* tf, double* rgba, orc_stats* st, int log_miss, int32_t* trace) {
    const int32_t W = fc->cam->width, H = fc->cam->height;
    const int nt = orc_get_threads();
    thread_acc* acc = (thread_acc*)calloc(nt, sizeof(thread_acc));
    int64_t rays = 0;
#pragma omp parallel reduction(+ : rays)
    {
#ifdef _OPENMP
        thread_acc* ta = &acc[omp_get_thread_num()];
#else
        thread_acc* ta = &acc[0];
#endif
#pragma omp for schedule(dynamic, 16)
        for (int64_t px = 0; px < (int64_t)W * H; ++px) {
            int32_t i = (int32_t)(px % W), j = (int32_t)(px / W);
            int32_t nproc = 0;
            render_pixel(fc, ta, tf, i, j, rgba + 4 * px, log_miss, &nproc);
            if (trace) trace[px] = nproc;
            float o[3], d[3], ts, te;
            if (orc_ray_setup(fc->cam, fc->m->dims, i, j, o, d, &ts, &te)) rays++;
        }
    }
    memset(st, 0, sizeof(*st));
    st->rays = rays;
    int64_t nm = 0;
    for (int t = 0; t < nt; ++t) {
        st->samples += acc[t].samples;
        st->hits += acc[t].hits;
        st->fallbacks += acc[t].fallbacks;
        st->misses += acc[t].misses;
        st->skipped += acc[t].skipped;
        st->ert_violations += acc[t].ert_violations;
        nm += acc[t].n_m;
    }
    if (fc->c) {
        orc_cache* c = fc->c;
        free(c->misses);
        c->misses = (miss_rec*)malloc(sizeof(miss_rec) * (nm ? nm : 1));
        c->n_misses = 0;
        for (int t = 0; t < nt; ++t) {
            memcpy(c->misses + c->n_misses, acc[t].misses_buf, sizeof(miss_rec) * acc[t].n_m);
            c->n_misses += acc[t].n_m;
        }
        qsort(c->misses, c->n_misses, sizeof(miss_rec), cmp_miss);
    }
    for (int t = 0; t < nt; ++t) free(acc[t].misses_buf);
    free(acc);
    return 0;
}

/* Per-cell flags (visible or not), or step codes with adaptive sampling. */
static uint8_t* make_flags(const orc_inr* m, const orc_params* p, const float* tf, int32_t M[3]) {
    if (p->macro_cell <= 0 || !p->macro_minmax) return NULL;
    for (int a = 0; a < 3; ++a) M[a] = (m->dims[a] + p->macro_cell - 1) / p->macro_cell;
    int64_t n = (int64_t)M[0] * M[1] * M[2];
    uint8_t* f = (uint8_t*)malloc(n);
    if (p->adapt_max_exp >= 0)
        orc_macrocell_step_codes(p->macro_minmax, n, tf, p->adapt_max_exp, f);
    else
        orc_macrocell_flags(p->macro_minmax, n, tf, f);
    return f;
}

int orc_render_uncached(const orc_inr* m, const orc_camera* c, const float* tf, const orc_params* p, double* rgba,
                        orc_stats* st) {
    if (p->mode != ORC_UNCACHED_DIRECT && p->mode != ORC_UNCACHED_LATTICE) return -1;
    if (!params_ok(p)) return -1;
    frame_ctx fc;
    memset(&fc, 0, sizeof(fc));
    fc.m = m;
    fc.cam = c;
    fc.p = p;
    for (int a = 0; a < 3; ++a) fc.vm1[a] = (float)(m->dims[a] - 1);
    fc.flags = make_flags(m, p, tf, fc.M);
    render_pass(&fc, tf, rgba, st, 0, NULL);
    free((void*)fc.flags);
    return 0;
}

typedef struct {
    int64_t rank;
    int32_t key;
} cand;

static int cmp_rank(const void* a, const void* b) {
    const cand* x = (const cand*)a;
    const cand* y = (const cand*)b;
    if (x->rank != y->rank) return x->rank > y->rank ? -1 : 1;
    return (x->key > y->key) - (x->key < y->key);
}

static int cmp_key(const void* a, const void* b) {
    const cand* x = (const cand*)a;
    const cand* y = (const cand*)b;
    return (x->key > y->key) - (x->key < y->key);
}

/* End of frame f (Section 4.3.3).  A brick requested c times in frame f gets
 * rank f + c - 1 the first time it is seen (timestamp of the first request,
 * plus one per further request) and rank + c afterwards; ranks are clamped to
 * f + rank_window.  The request list holds the top max_requests bricks
 * requested in this frame by (rank desc, key asc); the timestamp-only variant
 * takes them by key.  Counts are then cleared. */
static void end_of_frame(orc_cache* c, int32_t f, orc_stats* st) {
    cand* cs = (cand*)malloc(sizeof(cand) * (c->n_keys ? c->n_keys : 1));
    int64_t n = 0;
    for (int64_t k = 0; k < c->n_keys; ++k) {
        uint32_t cnt = c->req[k];
        c->last_req[k] = cnt;
        if (cnt == 0) continue;
        int64_t r = c->rank[k] < 0 ? (int64_t)f + (int64_t)cnt - 1 : c->rank[k] + (int64_t)cnt;
        if (r > (int64_t)f + c->d.rank_window) r = (int64_t)f + c->d.rank_window;
        c->rank[k] = r;
        cs[n].rank = r;
        cs[n].key = (int32_t)k;
        ++n;
        c->req[k] = 0;
    }
    qsort(cs, n, sizeof(cand), c->d.ranking ? cmp_rank : cmp_key);
    int64_t lim = c->d.max_requests < c->d.pool_bricks ? c->d.max_requests : c->d.pool_bricks;
    if (lim > n) lim = n;
    c->n_req_list = lim;
    for (int64_t i = 0; i < lim; ++i) c->req_list[i] = cs[i].key;
    st->requested = n;
    st->selected = lim;
    free(cs);
}

/* End of frame f: ranking and selection, then the insertion of the selected
 * bricks stamped f + 1 (they arrive at the start of the next frame). */
static void finish_frame(orc_cache* c, int32_t f, orc_stats* st) {
    end_of_frame(c, f, st);
    const int64_t ev0 = c->n_evlog;
    uint8_t* filled = (uint8_t*)calloc(c->d.pool_bricks > 0 ? c->d.pool_bricks : 1, 1);
    int32_t* slots = (int32_t*)malloc(sizeof(int32_t) * (size_t)(c->n_req_list > 0 ? c->n_req_list : 1));
    for (int64_t i = 0; i < c->n_req_list; ++i) insert_brick(c, c->req_list[i], f + 1, filled, &slots[i]);
    decode_inserted(c, c->req_list, slots, c->n_req_list);
    free(slots);
    free(filled);
    int64_t ev = 0;
    for (int64_t i = ev0; i < c->n_evlog; ++i)
        if (c->evlog[4 * i + 2] >= 0) ++ev;
    st->evicted = ev;
}

/* Scripted cache-manager scenarios: add request counts, stamp a slot as read
 * in a frame, or close a frame without rendering. */
int orc_cache_inject_requests(orc_cache* c, const int32_t* keys, const uint32_t* counts, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        if (keys[i] < 0 || keys[i] >= c->n_keys || c->pt[keys[i]] >= 0) return -1;
        c->req[keys[i]] += counts[i];
    }
    return 0;
}

int orc_cache_touch(orc_cache* c, int32_t slot, int32_t frame) {
    if (slot < 0 || slot >= c->d.pool_bricks) return -1;
    c->last_used[slot] = frame;
    return 0;
}

int orc_cache_end_frame(orc_cache* c, int32_t frame, orc_stats* st) {
    orc_stats tmp;
    memset(&tmp, 0, sizeof(tmp));
    finish_frame(c, frame, st ? st : &tmp);
    return 0;
}

int orc_cache_render(orc_cache* c, const orc_camera* cam, const float* tf, const orc_params* p, double* rgba,
                     orc_stats* st) {
    if (p->mode != ORC_CACHED) return -1;
    if (!params_ok(p)) return -1;
    frame_ctx fc;
    memset(&fc, 0, sizeof(fc));
    fc.m = &c->inr;
    fc.c = c;
    fc.cam = cam;
    fc.p = p;
    for (int a = 0; a < 3; ++a) fc.vm1[a] = (float)(c->inr.dims[a] - 1);
    fc.flags = make_flags(&c->inr, p, tf, fc.M);
    fc.frame_seed = orc_frame_seed(p->seed, (uint32_t)p->frame_index);
    fc.lod_floor = orc_lod_floor(p->frame_index, c->d.preload_period, c->d.n_lods);
    fc.preload = orc_preload_frame(p->frame_index, c->d.preload_period);
    int32_t* trace = NULL;
    if (c->trace_ert) {
        free(c->ert_trace);
        c->n_ert_trace = (int64_t)cam->width * cam->height;
        c->ert_trace = (int32_t*)malloc(sizeof(int32_t) * c->n_ert_trace);
        trace = c->ert_trace;
    }
    render_pass(&fc, tf, rgba, st, c->log_misses, trace);
    free((void*)fc.flags);
    finish_frame(c, p->frame_index, st);
    return 0;
}

/* One frame of several views through a shared cache: every view is rendered
 * against the residency at the start of the frame (its requests and stamps
 * accumulate), then one end-of-frame step ranks the requests of all views.
 * View i shows volume vol[i]; images are written to rgba + 4 * (sum of the
 * previous views' pixels); the miss list holds the misses of all views. */
int orc_cache_render_views(orc_cache* c, int32_t n, const int32_t* vol, const orc_camera* cams, const float* tfs,
                           const orc_params* ps, double* rgba, orc_stats* sts) {
    if (n < 1) return -1;
    for (int i = 0; i < n; ++i)
        if (ps[i].mode != ORC_CACHED || vol[i] < 0 || vol[i] >= c->n_vols || ps[i].frame_index != ps[0].frame_index ||
            !params_ok(&ps[i]))
            return -1;
    miss_rec* all = NULL;
    int64_t n_all = 0;
    double* out = rgba;
    for (int i = 0; i < n; ++i) {
        frame_ctx fc;
        memset(&fc, 0, sizeof(fc));
        fc.m = &c->inrs[vol[i]];
        fc.c = c;
        fc.key_base = (int64_t)vol[i] * c->keys_per_vol;
        fc.cam = &cams[i];
        fc.p = &ps[i];
        for (int a = 0; a < 3; ++a) fc.vm1[a] = (float)(fc.m->dims[a] - 1);
        fc.flags = make_flags(fc.m, &ps[i], tfs + 1024 * i, fc.M);
        fc.frame_seed = orc_frame_seed(ps[i].seed, (uint32_t)ps[i].frame_index);
        fc.lod_floor = orc_lod_floor(ps[i].frame_index, c->d.preload_period, c->d.n_lods);
        fc.preload = orc_preload_frame(ps[i].frame_index, c->d.preload_period);
        render_pass(&fc, tfs + 1024 * i, out, &sts[i], c->log_misses, NULL);
        free((void*)fc.flags);
        out += 4 * (int64_t)cams[i].width * cams[i].height;
        all = (miss_rec*)realloc(all, sizeof(miss_rec) * (size_t)(n_all + c->n_misses + 1));
        memcpy(all + n_all, c->misses, sizeof(miss_rec) * c->n_misses);
        n_all += c->n_misses;
    }
    free(c->misses);
    c->misses = all;
    c->n_misses = n_all;
    qsort(c->misses, c->n_misses, sizeof(miss_rec), cmp_miss);
    orc_stats fs;
    memset(&fs, 0, sizeof(fs));
    finish_frame(c, ps[0].frame_index, &fs);
    for (int i = 0; i < n; ++i) {
        sts[i].requested = fs.requested;
        sts[i].selected = fs.selected;
        sts[i].evicted = fs.evicted;
    }
    return 0;
}

/* Renders only the listed pixels (index j*W + i) of a frame, against the
 * cache's current residency (c may be NULL for the uncached modes), without
 * changing any cache state: no request counts, no stamps, no end of frame. */
int orc_render_pixels(const orc_inr* m, orc_cache* c, const orc_camera* cam, const float* tf, const orc_params* p,
                      const int32_t* pix, int64_t n, double* rgba) {
    if ((p->mode == ORC_CACHED) != (c != NULL)) return -1;
    if (!params_ok(p)) return -1;
    frame_ctx fc;
    memset(&fc, 0, sizeof(fc));
    fc.m = c ? &c->inr : m;
    fc.c = c;
    fc.readonly = 1;
    fc.cam = cam;
    fc.p = p;
    for (int a = 0; a < 3; ++a) fc.vm1[a] = (float)(fc.m->dims[a] - 1);
    fc.flags = make_flags(fc.m, p, tf, fc.M);
    if (c) {
        fc.frame_seed = orc_frame_seed(p->seed, (uint32_t)p->frame_index);
        fc.lod_floor = orc_lod_floor(p->frame_index, c->d.preload_period, c->d.n_lods);
        fc.preload = orc_preload_frame(p->frame_index, c->d.preload_period);
    }
    const int nt = orc_get_threads();
    thread_acc* acc = (thread_acc*)calloc(nt, sizeof(thread_acc));
#pragma omp parallel
    {
#ifdef _OPENMP
        thread_acc* ta = &acc[omp_get_thread_num()];
#else
        thread_acc* ta = &acc[0];
#endif
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < n; ++q) {
            const int32_t i = pix[q] % cam->width, j = pix[q] / cam->width;
            render_pixel(&fc, ta, tf, i, j, rgba + 4 * q, 0, NULL);
        }
    }
    for (int t = 0; t < nt; ++t) free(acc[t].misses_buf);
    free(acc);
    free((void*)fc.flags);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Learned part: MSE loss and analytic gradients, Adam                        */
/* ------------------------------------------------------------------------- */

/* Loss = mean over the batch of (y - target)^2 with y the raw network output
 * (training works on data normalised to [0,1], Section 4.1).  Gradients are
 * accumulated into g_table (same layout as the table) and g_weights. */
/* x rounded to binary32, then to bfloat16 (the upper 16 bits of a binary32:
 * 8 significant bits) to nearest, ties to even.  Infinities and NaNs are not
 * expected here. */
double orc_round_bf16(double x) {
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, sizeof b);
    b += 0x7FFFu + ((b >> 16) & 1u);
    b &= 0xFFFF0000u;
    memcpy(&f, &b, sizeof f);
    return (double)f;
}

double orc_loss_grad(const orc_inr* m, const double* u, const double* target, int64_t n, double* g_table,
                     double* g_weights) {
    return orc_loss_grad_prec(m, u, target, n, g_table, g_weights, 0);
}

/* With bf16_operands, every operand of the products of the hidden layers --
 * the encoded features, the activations entering a hidden layer, the weights
 * of the layers before the output layer and the back-propagated errors
 * leaving a ReLU -- is rounded by orc_round_bf16 before it is used (the
 * precision contract of a BF16 matrix-core MLP: BF16 operands, wider
 * accumulation); the output layer, the loss, the feature gradient and the
 * scatter into the table stay in FP64.  Otherwise everything is FP64. */
double orc_loss_grad_prec(const orc_inr* m, const double* u, const double* target, int64_t n, double* g_table,
                          double* g_weights, int bf16_operands) {
    const int F = m->n_features, NL = m->n_levels;
    const int64_t T = (int64_t)1 << m->log2_table;
    int64_t nw = 0;
    for (int k = 0; k < m->n_layers; ++k) nw += (int64_t)m->widths[k] * m->widths[k + 1];
    const int64_t ne = orc_table_entries(m);
    memset(g_table, 0, sizeof(double) * ne * F);
    memset(g_weights, 0, sizeof(double) * nw);
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double act[ORC_MAX_LAYERS + 1][256];
        double pre[ORC_MAX_LAYERS][256];
        encode_one(m, u + 3 * i, act[0]);
        const float* W = m->weights;
        for (int k = 0; k < m->n_layers; ++k) {
            const int ni = m->widths[k], no = m->widths[k + 1];
            const int q = bf16_operands && k + 1 < m->n_layers; /* a hidden layer's product */
            if (q)
                for (int cc = 0; cc < ni; ++cc) act[k][cc] = orc_round_bf16(act[k][cc]);
            for (int r = 0; r < no; ++r) {
                double s = 0.0;
                for (int cc = 0; cc < ni; ++cc) {
                    const double w = q ? orc_round_bf16((double)W[r * ni + cc]) : (double)W[r * ni + cc];
                    s += w * act[k][cc];
                }
                pre[k][r] = s;
                act[k + 1][r] = (k + 1 < m->n_layers && s < 0.0) ? 0.0 : s;
            }
            W += ni * no;
        }
        const double y = act[m->n_layers][0];
        const double e = y - target[i];
        loss += e * e;
        /* backward through the layers */
        double gout[256], gin[256];
        gout[0] = 2.0 * e / (double)n;
        int64_t woff = nw;
        for (int k = m->n_layers - 1; k >= 0; --k) {
            const int ni = m->widths[k], no = m->widths[k + 1];
            woff -= (int64_t)ni * no;
            const float* Wk = m->weights + woff;
            double* gW = g_weights + woff;
            const int q = bf16_operands && k + 1 < m->n_layers;
            for (int cc = 0; cc < ni; ++cc) gin[cc] = 0.0;
            for (int r = 0; r < no; ++r) {
                double gz = gout[r];
                if (k + 1 < m->n_layers && pre[k][r] < 0.0) gz = 0.0;
                if (q) gz = orc_round_bf16(gz);
                for (int cc = 0; cc < ni; ++cc) {
                    const double w = q ? orc_round_bf16((double)Wk[r * ni + cc]) : (double)Wk[r * ni + cc];
                    gW[r * ni + cc] += gz * act[k][cc];
                    gin[cc] += w * gz;
                }
            }
            for (int cc = 0; cc < ni; ++cc) gout[cc] = gin[cc];
        }
        /* gout now holds d loss / d feature; scatter into the grid corners */
        int64_t off = 0;
        for (int l = 0; l < NL; ++l) {
            const int64_t N = m->level_res[l];
            const int64_t side = N + 1;
            const int dense = side * side * side <= T;
            double w[3];
            int64_t c0[3];
            for (int a = 0; a < 3; ++a) {
                double s = u[3 * i + a] * (double)N;
                double fl = floor(s);
                c0[a] = (int64_t)fl;
                w[a] = s - fl;
            }
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
                        int64_t idx = grid_index(c0[0] + dx, c0[1] + dy, c0[2] + dz, side, dense, T);
                        for (int j = 0; j < F; ++j) g_table[(off + idx) * F + j] += wt * gout[l * F + j];
                    }
            off += orc_level_size(m, l);
        }
    }
    return loss / (double)n;
}

/* Uniform training points from a counter-based generator (one Philox block
 * per point; 24 bits per coordinate). */
void orc_train_points(uint64_t seed, int64_t step, int64_t n, double* u) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)step,
                                 (uint32_t)((uint64_t)step >> 32)};
        uint32_t r[4];
        orc_philox4x32_10(ctr, key, r);
        for (int a = 0; a < 3; ++a) u[3 * i + a] = (double)(r[a] >> 8) * (1.0 / 16777216.0);
    }
}

/* Trilinear interpolation of a voxel grid whose samples sit at cell centres
 * of the unit cube: position x = u * V - 0.5 in voxel units, clamped to the
 * sample range; the cell is clamped so that its upper corner exists. */
void orc_grid_trilinear(const float* grid, const int32_t dims[3], const double* u, int64_t n, double* out) {
    const int64_t sx = 1, sy = dims[0], sz = (int64_t)dims[0] * dims[1];
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        double f[3];
        for (int a = 0; a < 3; ++a) {
            double x = u[3 * i + a] * (double)dims[a] - 0.5;
            if (x < 0.0) x = 0.0;
            if (x > (double)(dims[a] - 1)) x = (double)(dims[a] - 1);
            int64_t j = (int64_t)floor(x);
            if (j > dims[a] - 2) j = dims[a] - 2;
            if (j < 0) j = 0;
            c[a] = j;
            f[a] = dims[a] > 1 ? x - (double)j : 0.0;
        }
        const float* g = grid + c[2] * sz + c[1] * sy + c[0] * sx;
        const int64_t dx = dims[0] > 1 ? sx : 0, dy = dims[1] > 1 ? sy : 0, dz = dims[2] > 1 ? sz : 0;
        double v = 0.0;
        for (int k = 0; k < 8; ++k) {
            const int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
            const double w = (bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) * (bz ? f[2] : 1.0 - f[2]);
            v += w * (double)g[bx * dx + by * dy + bz * dz];
        }
        out[i] = v;
    }
}

/* Adam (Kingma and Ba 2015) with bias correction; `step` counts from 1. */
void orc_adam_step(double* p, double* m1, double* m2, const double* g, int64_t n, int64_t step, double lr, double b1,
                   double b2, double eps) {
    const double c1 = 1.0 - pow(b1, (double)step);
    const double c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        m1[i] = b1 * m1[i] + (1.0 - b1) * g[i];
        m2[i] = b2 * m2[i] + (1.0 - b2) * g[i] * g[i];
        const double mh = m1[i] / c1;
        const double vh = m2[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
