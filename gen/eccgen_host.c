/*
 * Seeded synthetic image generators, host side.
 *
 * This module only produces input bytes. It contains none of the Euler
 * characteristic arithmetic, and it is shared by the CPU oracle (tests) and the
 * GPU benchmarks, which both read what it writes.
 *
 * Random source: a counter-based hash built from SplitMix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
 *
 *   mix64(z)          = z ^= z>>30; z *= 0xBF58476D1CE4E5B9;
 *                       z ^= z>>27; z *= 0x94D049BB133111EB; z ^ (z>>31)
 *   key(seed, stream) = mix64(seed * GAMMA + stream)          (mod 2^64)
 *   h(seed, stream, i)= mix64(key(seed, stream) + (i + 1) * GAMMA)
 *
 * with GAMMA = 0x9E3779B97F4A7C15, i.e. h(.,.,i) is output number i of a
 * SplitMix64 sequence whose state starts at key(seed, stream).
 *
 * Families (stream 0: i.i.d. values, 1: lattice values, 2: per-voxel jitter):
 *   iid:          v[i] = h(seed, 0, i) >> (64 - bits)
 *   value noise:  lattice spacing L = 2^lshift on every axis, node grid
 *                 N_k = ((n_k - 1) >> lshift) + 2 nodes per axis (C order),
 *                 U(node) = h(seed, 1, node_linear) >> (64 - bits);
 *                 d-linear integer interpolation with weights (L - r_k) and
 *                 r_k, r_k = p_k mod L, total weight L^d, rounded half up:
 *                 base = (sum + L^d/2) >> (d * lshift);
 *                 jitter J = (((h(seed, 2, i) >> 32) * (2A + 1)) >> 32) - A,
 *                 uniform on the integers [-A, A];
 *                 v = clamp(base + J, 0, 2^bits - 1).
 *   float noise:  U(node) = (h(seed, 1, node_linear) >> 40) * 2^-24 in [0,1),
 *                 d-linear interpolation in double with weights (L-r)/L, r/L,
 *                 plus sigma * z, z standard normal by Box-Muller from
 *                 h = h(seed, 2, i): u1 = ((h >> 32) + 1) * 2^-32,
 *                 u2 = (h & 0xffffffff) * 2^-32, z = sqrt(-2 ln u1) cos(2 pi u2);
 *                 stored as the float32 nearest to the double.
 * i is the C-order linear index of the voxel in the whole image.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL
#define MAXD 8

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t eccgen_key(uint64_t seed, uint64_t stream) { return mix64(seed * GAMMA + stream); }

uint64_t eccgen_hash(uint64_t seed, uint64_t stream, uint64_t i) {
    return mix64(eccgen_key(seed, stream) + (i + 1) * GAMMA);
}

/* ---------------------------------------------------------------- threads */
typedef struct {
    void (*fn)(void *ctx, int64_t lo, int64_t hi);
    void *ctx;
    int64_t lo, hi;
} span_t;

static void *span_run(void *p) {
    span_t *s = (span_t *)p;
    s->fn(s->ctx, s->lo, s->hi);
    return NULL;
}

static void parallel_for(int64_t count, int nthreads, void (*fn)(void *, int64_t, int64_t), void *ctx) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > count) nthreads = (int)(count > 0 ? count : 1);
    if (nthreads == 1) { fn(ctx, 0, count); return; }
    pthread_t th[256];
    span_t sp[256];
    for (int t = 0; t < nthreads; ++t) {
        sp[t].fn = fn; sp[t].ctx = ctx;
        sp[t].lo = count * t / nthreads;
        sp[t].hi = count * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, span_run, &sp[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------- iid */
typedef struct { uint64_t key; int shift; int64_t start; void *out; int elem; } iid_ctx;

static void iid_body(void *p, int64_t lo, int64_t hi) {
    iid_ctx *c = (iid_ctx *)p;
    for (int64_t j = lo; j < hi; ++j) {
        uint64_t v = mix64(c->key + (uint64_t)(c->start + j + 1) * GAMMA) >> c->shift;
        if (c->elem == 1) ((uint8_t *)c->out)[j] = (uint8_t)v;
        else ((uint16_t *)c->out)[j] = (uint16_t)v;
    }
}

/* out[j] = h(seed, 0, start + j) >> (64 - bits), j in [0, count). elem = 1 or 2 bytes. */
int eccgen_iid(uint64_t seed, int bits, int64_t start, int64_t count, void *out, int elem, int nthreads) {
    if (bits < 1 || bits > 8 * elem || (elem != 1 && elem != 2) || count < 0) return -1;
    iid_ctx c = {eccgen_key(seed, 0), 64 - bits, start, out, elem};
    parallel_for(count, nthreads, iid_body, &c);
    return 0;
}

/* ----------------------------------------------------------- value noise */
typedef struct {
    int d, lshift, bits, amp, elem, is_float;
    int64_t n[MAXD], N[MAXD];
    int64_t z0;                 /* first generated plane of axis 0 */
    uint64_t key1, key2;
    double sigma;
    void *out;
    int64_t plane;              /* voxels per axis-0 plane */
} vn_ctx;

static void vn_body(void *p, int64_t lo, int64_t hi) {
    vn_ctx *c = (vn_ctx *)p;
    const int d = c->d, ls = c->lshift;
    const int64_t L = (int64_t)1 << ls;
    const int64_t maxv = ((int64_t)1 << c->bits) - 1;
    int64_t coord[MAXD];
    /* lo..hi index voxels of the generated range, C order */
    for (int64_t j = lo; j < hi; ++j) {
        int64_t rem = j % c->plane;
        coord[0] = c->z0 + j / c->plane;
        for (int k = d - 1; k >= 1; --k) {
            coord[k] = rem % c->n[k];
            rem /= c->n[k];
        }
        int64_t gidx = 0;
        for (int k = 0; k < d; ++k) gidx = gidx * c->n[k] + coord[k];
        int64_t base[MAXD], r[MAXD];
        for (int k = 0; k < d; ++k) { base[k] = coord[k] >> ls; r[k] = coord[k] & (L - 1); }
        if (!c->is_float) {
            uint64_t acc = 0;
            for (int corner = 0; corner < (1 << d); ++corner) {
                uint64_t w = 1;
                int64_t node = 0;
                for (int k = 0; k < d; ++k) {
                    int bit = (corner >> (d - 1 - k)) & 1;
                    node = node * c->N[k] + base[k] + bit;
                    w *= (uint64_t)(bit ? r[k] : (L - r[k]));
                }
                uint64_t u = mix64(c->key1 + (uint64_t)(node + 1) * GAMMA) >> (64 - c->bits);
                acc += u * w;
            }
            int64_t bv = (int64_t)((acc + ((uint64_t)1 << (d * ls - 1))) >> (d * ls));
            uint64_t hj = mix64(c->key2 + (uint64_t)(gidx + 1) * GAMMA);
            int64_t jit = (int64_t)(((hj >> 32) * (uint64_t)(2 * c->amp + 1)) >> 32) - c->amp;
            int64_t v = bv + jit;
            if (v < 0) v = 0;
            if (v > maxv) v = maxv;
            if (c->elem == 1) ((uint8_t *)c->out)[j] = (uint8_t)v;
            else ((uint16_t *)c->out)[j] = (uint16_t)v;
        } else {
            double acc = 0.0;
            for (int corner = 0; corner < (1 << d); ++corner) {
                double w = 1.0;
                int64_t node = 0;
                for (int k = 0; k < d; ++k) {
                    int bit = (corner >> (d - 1 - k)) & 1;
                    node = node * c->N[k] + base[k] + bit;
                    w *= bit ? (double)r[k] / (double)L : (double)(L - r[k]) / (double)L;
                }
                uint64_t u = mix64(c->key1 + (uint64_t)(node + 1) * GAMMA) >> 40;
                acc += (double)u * (1.0 / 16777216.0) * w;
            }
            uint64_t hj = mix64(c->key2 + (uint64_t)(gidx + 1) * GAMMA);
            double u1 = ((double)(hj >> 32) + 1.0) * (1.0 / 4294967296.0);
            double u2 = (double)(hj & 0xffffffffULL) * (1.0 / 4294967296.0);
            double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
            ((float *)c->out)[j] = (float)(acc + c->sigma * z);
        }
    }
}

static int vn_setup(vn_ctx *c, uint64_t seed, int d, const int64_t *dims, int lshift, int64_t z0, int64_t z1) {
    if (d < 1 || d > MAXD || lshift < 1 || lshift > 8) return -1;
    c->d = d; c->lshift = lshift; c->z0 = z0;
    c->plane = 1;
    for (int k = 0; k < d; ++k) {
        if (dims[k] < 1) return -1;
        c->n[k] = dims[k];
        c->N[k] = ((dims[k] - 1) >> lshift) + 2;
        if (k > 0) c->plane *= dims[k];
    }
    if (z0 < 0 || z1 < z0 || z1 > dims[0]) return -1;
    c->key1 = eccgen_key(seed, 1);
    c->key2 = eccgen_key(seed, 2);
    return 0;
}

/* The same integer value noise for d = 3, one image row (fixed axis-0 and
 * axis-1 coordinates) at a time: the lattice values a row touches are hashed
 * once per row and node column instead of once per voxel and corner, and the
 * two outer interpolation weights are folded into one column sum
 * C[b] = sum_{i,j} w0(i) w1(j) U(b0+i, b1+j, b), so that
 * sum = (L - r2) C[b2] + r2 C[b2+1].  Every term is an exact integer, so the
 * sum, and every output byte, equals the per-voxel form above. */
static void vn_rows3(void *p, int64_t lo, int64_t hi) {
    vn_ctx *c = (vn_ctx *)p;
    const int ls = c->lshift;
    const int64_t L = (int64_t)1 << ls;
    const int64_t maxv = ((int64_t)1 << c->bits) - 1;
    const int64_t n1 = c->n[1], n2 = c->n[2], N1 = c->N[1], N2 = c->N[2];
    uint64_t *col = (uint64_t *)malloc((size_t)N2 * sizeof(uint64_t));
    if (!col) return;  /* out of memory: rows stay unwritten (callers size this to a few KiB) */
    for (int64_t row = lo; row < hi; ++row) {
        const int64_t z = c->z0 + row / n1, y = row % n1;
        const int64_t b0 = z >> ls, r0 = z & (L - 1), b1 = y >> ls, r1 = y & (L - 1);
        for (int64_t b = 0; b < N2; ++b) {
            uint64_t s = 0;
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    const int64_t node = ((b0 + i) * N1 + (b1 + j)) * N2 + b;
                    const uint64_t u = mix64(c->key1 + (uint64_t)(node + 1) * GAMMA) >> (64 - c->bits);
                    s += u * (uint64_t)((i ? r0 : L - r0) * (j ? r1 : L - r1));
                }
            col[b] = s;
        }
        const int64_t gbase = (z * n1 + y) * n2;
        const int64_t obase = row * n2;
        for (int64_t x = 0; x < n2; ++x) {
            const int64_t b2 = x >> ls, r2 = x & (L - 1);
            const uint64_t acc = (uint64_t)(L - r2) * col[b2] + (uint64_t)r2 * col[b2 + 1];
            const int64_t bv = (int64_t)((acc + ((uint64_t)1 << (3 * ls - 1))) >> (3 * ls));
            const uint64_t hj = mix64(c->key2 + (uint64_t)(gbase + x + 1) * GAMMA);
            int64_t v = bv + (int64_t)(((hj >> 32) * (uint64_t)(2 * c->amp + 1)) >> 32) - c->amp;
            if (v < 0) v = 0;
            if (v > maxv) v = maxv;
            if (c->elem == 1) ((uint8_t *)c->out)[obase + x] = (uint8_t)v;
            else ((uint16_t *)c->out)[obase + x] = (uint16_t)v;
        }
    }
    free(col);
}

/* The d = 2 row form: one row (fixed axis-0 coordinate) at a time, the
 * lattice values of its two node rows hashed once per node column and folded
 * into C[b] = sum_i w0(i) U(b0+i, b); sum = (L - r1) C[b1] + r1 C[b1+1]. */
static void vn_rows2(void *p, int64_t lo, int64_t hi) {
    vn_ctx *c = (vn_ctx *)p;
    const int ls = c->lshift;
    const int64_t L = (int64_t)1 << ls;
    const int64_t maxv = ((int64_t)1 << c->bits) - 1;
    const int64_t n1 = c->n[1], N1 = c->N[1];
    uint64_t *col = (uint64_t *)malloc((size_t)N1 * sizeof(uint64_t));
    if (!col) return;
    for (int64_t row = lo; row < hi; ++row) {
        const int64_t z = c->z0 + row;
        const int64_t b0 = z >> ls, r0 = z & (L - 1);
        for (int64_t b = 0; b < N1; ++b) {
            uint64_t s = 0;
            for (int i = 0; i < 2; ++i) {
                const int64_t node = (b0 + i) * N1 + b;
                const uint64_t u = mix64(c->key1 + (uint64_t)(node + 1) * GAMMA) >> (64 - c->bits);
                s += u * (uint64_t)(i ? r0 : L - r0);
            }
            col[b] = s;
        }
        for (int64_t x = 0; x < n1; ++x) {
            const int64_t b1 = x >> ls, r1 = x & (L - 1);
            const uint64_t acc = (uint64_t)(L - r1) * col[b1] + (uint64_t)r1 * col[b1 + 1];
            const int64_t bv = (int64_t)((acc + ((uint64_t)1 << (2 * ls - 1))) >> (2 * ls));
            const uint64_t hj = mix64(c->key2 + (uint64_t)(z * n1 + x + 1) * GAMMA);
            int64_t v = bv + (int64_t)(((hj >> 32) * (uint64_t)(2 * c->amp + 1)) >> 32) - c->amp;
            if (v < 0) v = 0;
            if (v > maxv) v = maxv;
            if (c->elem == 1) ((uint8_t *)c->out)[row * n1 + x] = (uint8_t)v;
            else ((uint16_t *)c->out)[row * n1 + x] = (uint16_t)v;
        }
    }
    free(col);
}

/* Integer value noise for planes [z0, z1) of axis 0; out holds (z1-z0)*plane values. */
int eccgen_value_noise(uint64_t seed, int d, const int64_t *dims, int lshift, int bits, int amp,
                       int64_t z0, int64_t z1, void *out, int elem, int nthreads) {
    vn_ctx c;
    memset(&c, 0, sizeof c);
    if (vn_setup(&c, seed, d, dims, lshift, z0, z1)) return -1;
    if ((elem != 1 && elem != 2) || bits < 1 || bits > 8 * elem || amp < 0) return -1;
    if (d * lshift + bits > 60) return -1;
    c.bits = bits; c.amp = amp; c.elem = elem; c.is_float = 0; c.out = out;
    if (d == 3)
        parallel_for((z1 - z0) * c.n[1], nthreads, vn_rows3, &c);
    else if (d == 2)
        parallel_for(z1 - z0, nthreads, vn_rows2, &c);
    else
        parallel_for((z1 - z0) * c.plane, nthreads, vn_body, &c);
    return 0;
}

/* The per-voxel form for any d (the d = 3 row form above is checked against it). */
int eccgen_value_noise_voxelwise(uint64_t seed, int d, const int64_t *dims, int lshift, int bits, int amp,
                                 int64_t z0, int64_t z1, void *out, int elem, int nthreads) {
    vn_ctx c;
    memset(&c, 0, sizeof c);
    if (vn_setup(&c, seed, d, dims, lshift, z0, z1)) return -1;
    if ((elem != 1 && elem != 2) || bits < 1 || bits > 8 * elem || amp < 0) return -1;
    if (d * lshift + bits > 60) return -1;
    c.bits = bits; c.amp = amp; c.elem = elem; c.is_float = 0; c.out = out;
    parallel_for((z1 - z0) * c.plane, nthreads, vn_body, &c);
    return 0;
}

/* Float value noise with Gaussian jitter of standard deviation sigma. */
int eccgen_value_noise_f32(uint64_t seed, int d, const int64_t *dims, int lshift, double sigma,
                           int64_t z0, int64_t z1, float *out, int nthreads) {
    vn_ctx c;
    memset(&c, 0, sizeof c);
    if (vn_setup(&c, seed, d, dims, lshift, z0, z1)) return -1;
    c.is_float = 1; c.sigma = sigma; c.out = out; c.bits = 24;
    parallel_for((z1 - z0) * c.plane, nthreads, vn_body, &c);
    return 0;
}
