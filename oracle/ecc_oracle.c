/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow CPU computation of the Euler characteristic curve of a
 * d-dimensional gray-scale image, written straight from the definitions of
 * Heiss & Wagner, "Streaming Algorithm for Euler Characteristic Curves of
 * Multidimensional Images" (arXiv 1705.02045), Section 2:
 *
 *  - Cubical cell (Sec. 2, "Cubical Cell"): a product of d factors, each an
 *    interval [a, a+1] or a singleton {b}; its dimension is the number of
 *    interval factors.  We index cells by doubled coordinates q in
 *    prod_k [0, 2 n_k]: odd q_k = 2a+1 is the interval [a, a+1], even
 *    q_k = 2b is the singleton {b}.
 *  - Image as a complex (Sec. 2, "Consecutive Thresholded Images as Sublevel
 *    Set Filtrations"): voxel (i_1..i_d) is the d-cell prod [i_k - 1, i_k]
 *    (1-based in the paper; 0-based here, voxel a is [a, a+1]); K is the set of
 *    all voxel cells and all their faces.  Every q above is a cell of K.
 *  - Sublevel set filtration (Sec. 2, "Sublevel Set Filtration"): a cell's
 *    value is the minimum of f over the voxels (maximal cells) containing it.
 *    Those voxels are prod_k I_k with I_k = {a} for odd q_k and
 *    I_k = {b-1, b} intersected with [0, n_k) for even q_k.
 *  - Euler characteristic (Sec. 2, "Euler Characteristic"):
 *    chi = sum_k (-1)^k n_k.
 *  - VCEC (Sec. 3, "Tracking the Changes"): a_t = chi(T_t) - chi(T_{t-1}),
 *    which is the signed count of cells whose value is exactly t; the curve
 *    is its prefix sum (Sec. 3, "Post-Processing").
 *
 * Nothing here uses the paper's per-voxel "introduced faces" rule: every cell
 * is visited once and its value is computed from its incident voxels.  Threads
 * only split the cells by ranges of the first doubled coordinate, each thread
 * into a private int64 array, and the arrays are summed at the end.
 *
 * Element types: 1 = uint8, 2 = uint16, 4 = uint32.  Every value must be < m.
 *
 * Dual complex (oracle_curve_dual; the construction the paper's footnote
 * to Sec. 2 "Consecutive Thresholded Images" sets against its own, with
 * voxels as vertices): the vertices are the voxels, and a cell is a product
 * of factors each either one voxel index {a} or a pair {a, a+1} of
 * neighbours along that axis -- doubled coordinates p in prod_k
 * [0, 2 (n_k - 1)], even p_k = 2a the index a, odd p_k = 2a+1 the pair;
 * dimension = number of pairs.  A cell enters when all its vertices have
 * (lower-star filtration): value = MAXIMUM of f over its vertices.  Edges join
 * voxels that share a (d-1)-face only (2d-connectivity).
 *
 * Second convention (the *_max entry points): a cell's value is the MAXIMUM
 * of f over the voxels containing it -- the literal "largest gray value among
 * its voxels" reading of the entry value, the alternative to Sec. 2's
 * minimum.  Its cell sets are not complexes (a face can enter after a cell it
 * bounds), so the "curve" is the signed cell count sum_{c: value(c) <= t}
 * (-1)^dim c, computed the same way with max in place of min.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 8

typedef struct {
    const void *img;
    int elem, d;
    int64_t n[MAXD], stride[MAXD];
    int64_t m;
    int64_t q0_lo, q0_hi;
    int use_max;                /* 0: minimum over incident voxels, 1: maximum */
    int dual;                   /* 1: cells of the dual complex (voxels as vertices) */
    int64_t *vcec;
} job_t;

static inline uint64_t load(const void *img, int elem, int64_t i) {
    switch (elem) {
    case 1: return ((const uint8_t *)img)[i];
    case 2: return ((const uint16_t *)img)[i];
    default: return ((const uint32_t *)img)[i];
    }
}

/* Adds the signed count of every cell with first doubled coordinate in
 * [q0_lo, q0_hi) into vcec[value]. */
static void count_cells(const job_t *j) {
    const int d = j->d;
    int64_t q[MAXD], lo[MAXD], hi[MAXD], idx[MAXD];
    for (int64_t q0 = j->q0_lo; q0 < j->q0_hi; ++q0) {
        q[0] = q0;
        for (int k = 1; k < d; ++k) q[k] = 0;
        for (;;) {
            /* incident voxels and dimension of cell q */
            int dim = 0;
            for (int k = 0; k < d; ++k) {
                if (j->dual) {  /* even: one voxel; odd: the pair (a, a+1) */
                    lo[k] = q[k] / 2;
                    hi[k] = (q[k] + 1) / 2;
                    dim += (int)(q[k] & 1);
                } else if (q[k] & 1) {
                    lo[k] = hi[k] = (q[k] - 1) / 2;
                    ++dim;
                } else {
                    int64_t b = q[k] / 2;
                    lo[k] = b - 1 < 0 ? 0 : b - 1;
                    hi[k] = b > j->n[k] - 1 ? j->n[k] - 1 : b;
                }
            }
            /* minimum (or maximum) of f over the incident voxels */
            uint64_t best = j->use_max ? 0 : UINT64_MAX;
            for (int k = 0; k < d; ++k) idx[k] = lo[k];
            for (;;) {
                int64_t lin = 0;
                for (int k = 0; k < d; ++k) lin += idx[k] * j->stride[k];
                uint64_t v = load(j->img, j->elem, lin);
                if (j->use_max ? v > best : v < best) best = v;
                int k = d - 1;
                while (k >= 0 && idx[k] == hi[k]) { idx[k] = lo[k]; --k; }
                if (k < 0) break;
                ++idx[k];
            }
            j->vcec[best] += (dim & 1) ? -1 : 1;
            /* next cell in this q0 layer */
            int k = d - 1;
            while (k >= 1 && q[k] == 2 * j->n[k] - (j->dual ? 2 : 0)) { q[k] = 0; --k; }
            if (k < 1) break;
            ++q[k];
        }
    }
}

static void *run_job(void *p) {
    count_cells((const job_t *)p);
    return NULL;
}

static int setup(job_t *base, const void *img, int elem, int d, const int64_t *n, int64_t m) {
    if (!img || d < 1 || d > MAXD || m < 1 || (elem != 1 && elem != 2 && elem != 4)) return -1;
    int64_t total = 1;
    for (int k = d - 1; k >= 0; --k) {
        if (n[k] < 1) return -1;
        base->n[k] = n[k];
        base->stride[k] = total;
        total *= n[k];
    }
    for (int64_t i = 0; i < total; ++i)
        if (load(img, elem, i) >= (uint64_t)m) return -2;
    base->img = img; base->elem = elem; base->d = d; base->m = m;
    return 0;
}

/* Signed cell counts for cells with q_0 in [q0_lo, q0_hi), added into vcec[0..m). */
int oracle_vcec_range(const void *img, int elem, int d, const int64_t *n, int64_t m,
                      int64_t q0_lo, int64_t q0_hi, int64_t *vcec) {
    job_t j;
    memset(&j, 0, sizeof j);
    int rc = setup(&j, img, elem, d, n, m);
    if (rc) return rc;
    if (q0_lo < 0) q0_lo = 0;
    if (q0_hi > 2 * n[0] + 1) q0_hi = 2 * n[0] + 1;
    j.q0_lo = q0_lo; j.q0_hi = q0_hi; j.vcec = vcec;
    if (q0_lo < q0_hi) count_cells(&j);
    return 0;
}

static int vcec_rule(const void *img, int elem, int d, const int64_t *n, int64_t m, int use_max, int dual,
                     int64_t *vcec, int nthreads, int64_t max_bytes) {
    job_t base;
    memset(&base, 0, sizeof base);
    int rc = setup(&base, img, elem, d, n, m);
    if (rc) return rc;
    base.use_max = use_max;
    base.dual = dual;
    int64_t layers = dual ? 2 * n[0] - 1 : 2 * n[0] + 1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > layers) nthreads = (int)layers;
    if (max_bytes > 0) {
        int64_t cap = max_bytes / (m * (int64_t)sizeof(int64_t));
        if (cap < 1) cap = 1;
        if (nthreads > cap) nthreads = (int)cap;
    }
    memset(vcec, 0, (size_t)m * sizeof(int64_t));
    if (nthreads == 1) {
        base.q0_lo = 0; base.q0_hi = layers; base.vcec = vcec;
        count_cells(&base);
        return 0;
    }
    job_t jobs[256];
    pthread_t th[256];
    int64_t *priv = (int64_t *)calloc((size_t)m * (size_t)nthreads, sizeof(int64_t));
    if (!priv) return -3;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].q0_lo = layers * t / nthreads;
        jobs[t].q0_hi = layers * (t + 1) / nthreads;
        jobs[t].vcec = priv + (size_t)m * t;
        pthread_create(&th[t], NULL, run_job, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < nthreads; ++t)
        for (int64_t s = 0; s < m; ++s) vcec[s] += priv[(size_t)m * t + s];
    free(priv);
    return 0;
}

/* VCEC of the whole image with up to nthreads threads.  Thread count is
 * lowered so that the private arrays stay within max_bytes. */
int oracle_vcec(const void *img, int elem, int d, const int64_t *n, int64_t m,
                int64_t *vcec, int nthreads, int64_t max_bytes) {
    return vcec_rule(img, elem, d, n, m, 0, 0, vcec, nthreads, max_bytes);
}

/* The curve chi(T_t), t = 0..m-1: prefix sums of the VCEC. */
int oracle_curve(const void *img, int elem, int d, const int64_t *n, int64_t m,
                 int64_t *chi, int nthreads, int64_t max_bytes) {
    int rc = oracle_vcec(img, elem, d, n, m, chi, nthreads, max_bytes);
    if (rc) return rc;
    for (int64_t t = 1; t < m; ++t) chi[t] += chi[t - 1];
    return 0;
}

/* The same with each cell's value the maximum over its voxels. */
int oracle_curve_max(const void *img, int elem, int d, const int64_t *n, int64_t m,
                     int64_t *chi, int nthreads, int64_t max_bytes) {
    int rc = vcec_rule(img, elem, d, n, m, 1, 0, chi, nthreads, max_bytes);
    if (rc) return rc;
    for (int64_t t = 1; t < m; ++t) chi[t] += chi[t - 1];
    return 0;
}

/* Curve of the dual complex (voxels as vertices, value = max over vertices). */
int oracle_curve_dual(const void *img, int elem, int d, const int64_t *n, int64_t m,
                      int64_t *chi, int nthreads, int64_t max_bytes) {
    int rc = vcec_rule(img, elem, d, n, m, 1, 1, chi, nthreads, max_bytes);
    if (rc) return rc;
    for (int64_t t = 1; t < m; ++t) chi[t] += chi[t - 1];
    return 0;
}

/* ------------------------------------------------------------------------
 * The same cell enumeration written out for d = 3 (three nested loops over
 * the doubled coordinates), for the large volumes whose curves are stored as
 * test fixtures.  It computes exactly what oracle_vcec_range computes for a
 * 3-D image -- every cell with q_0 in [q0_lo, q0_hi), its value the minimum
 * of f over its incident voxels, (-1)^dim added there (Sec. 2, "Sublevel Set
 * Filtration"; Sec. 3, "Tracking the Changes") -- with the incident-voxel
 * ranges computed per axis instead of by the d-dimensional odometer.  Threads
 * split the q_0 layers, each into a private array; the arrays are added into
 * vcec (which is not cleared). */
typedef struct {
    const void *img;
    int elem;
    int64_t n0, n1, n2, m;
    int64_t q0_lo, q0_hi;
    int64_t *vcec;
} job3_t;

/* incident index range {a} (odd q) or {b-1, b} within [0, n) (even q = 2b) */
static inline void incident(int64_t q, int64_t n, int64_t *lo, int64_t *hi) {
    if (q & 1) {
        *lo = *hi = (q - 1) / 2;
    } else {
        const int64_t b = q / 2;
        *lo = b - 1 < 0 ? 0 : b - 1;
        *hi = b > n - 1 ? n - 1 : b;
    }
}

/* One loop nest per element type (T), so that each voxel read is a plain
 * array access. */
#define COUNT_CELLS3(NAME, T)                                                        \
    static void NAME(const job3_t *j) {                                             \
        const T *f = (const T *)j->img;                                             \
        const int64_t n0 = j->n0, n1 = j->n1, n2 = j->n2;                           \
        for (int64_t q0 = j->q0_lo; q0 < j->q0_hi; ++q0) {                          \
            int64_t z0, z1;                                                         \
            incident(q0, n0, &z0, &z1);                                             \
            for (int64_t q1 = 0; q1 <= 2 * n1; ++q1) {                              \
                int64_t y0, y1;                                                     \
                incident(q1, n1, &y0, &y1);                                         \
                for (int64_t q2 = 0; q2 <= 2 * n2; ++q2) {                          \
                    int64_t x0, x1;                                                 \
                    incident(q2, n2, &x0, &x1);                                     \
                    T best = f[(z0 * n1 + y0) * n2 + x0];                           \
                    for (int64_t z = z0; z <= z1; ++z)                              \
                        for (int64_t y = y0; y <= y1; ++y)                          \
                            for (int64_t x = x0; x <= x1; ++x) {                    \
                                const T v = f[(z * n1 + y) * n2 + x];               \
                                if (v < best) best = v;                             \
                            }                                                       \
                    const int dim = (int)((q0 & 1) + (q1 & 1) + (q2 & 1));          \
                    j->vcec[best] += (dim & 1) ? -1 : 1;                            \
                }                                                                   \
            }                                                                       \
        }                                                                           \
    }
COUNT_CELLS3(count_cells3_u8, uint8_t)
COUNT_CELLS3(count_cells3_u16, uint16_t)
COUNT_CELLS3(count_cells3_u32, uint32_t)
#undef COUNT_CELLS3

static void count_cells3(const job3_t *j) {
    if (j->elem == 1) count_cells3_u8(j);
    else if (j->elem == 2) count_cells3_u16(j);
    else count_cells3_u32(j);
}

static void *run_job3(void *p) {
    count_cells3((const job3_t *)p);
    return NULL;
}

/* Signed counts of the cells with q_0 in [q0_lo, q0_hi) of a 3-D image
 * (dims n[0..2]), added into vcec[0..m), on up to nthreads threads.
 * Returns -1 on bad arguments, -2 if a value is >= m, -3 if out of memory. */
int oracle_vcec3(const void *img, int elem, const int64_t *n, int64_t m, int64_t q0_lo, int64_t q0_hi,
                 int64_t *vcec, int nthreads) {
    job_t chk;
    memset(&chk, 0, sizeof chk);
    int rc = setup(&chk, img, elem, 3, n, m);
    if (rc) return rc;
    if (q0_lo < 0) q0_lo = 0;
    if (q0_hi > 2 * n[0] + 1) q0_hi = 2 * n[0] + 1;
    if (q0_lo >= q0_hi) return 0;
    const int64_t layers = q0_hi - q0_lo;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > layers) nthreads = (int)layers;
    job3_t base = {img, elem, n[0], n[1], n[2], m, q0_lo, q0_hi, vcec};
    if (nthreads == 1) {
        count_cells3(&base);
        return 0;
    }
    job3_t jobs[256];
    pthread_t th[256];
    int64_t *priv = (int64_t *)calloc((size_t)m * (size_t)nthreads, sizeof(int64_t));
    if (!priv) return -3;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].q0_lo = q0_lo + layers * t / nthreads;
        jobs[t].q0_hi = q0_lo + layers * (t + 1) / nthreads;
        jobs[t].vcec = priv + (size_t)m * t;
        pthread_create(&th[t], NULL, run_job3, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < nthreads; ++t)
        for (int64_t s = 0; s < m; ++s) vcec[s] += priv[(size_t)m * t + s];
    free(priv);
    return 0;
}
