/*
 * Test driver for sanitizer builds of the oracle (test infrastructure only):
 * runs every entry point of ecc_oracle.c on small seeded images, single- and
 * multi-threaded, and checks the three-loop 3-D enumeration against the
 * general one and chi at the top threshold (1: the full box is
 * contractible).  Built by tests/test_oracle_sanitizers.py with
 * -fsanitize=address,undefined and with -fsanitize=thread; exits non-zero on
 * a mismatch, the sanitizers on any error they find.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_vcec(const void *img, int elem, int d, const int64_t *n, int64_t m, int64_t *vcec, int nthreads,
                int64_t max_bytes);
int oracle_curve(const void *img, int elem, int d, const int64_t *n, int64_t m, int64_t *chi, int nthreads,
                 int64_t max_bytes);
int oracle_curve_max(const void *img, int elem, int d, const int64_t *n, int64_t m, int64_t *chi, int nthreads,
                     int64_t max_bytes);
int oracle_curve_dual(const void *img, int elem, int d, const int64_t *n, int64_t m, int64_t *chi, int nthreads,
                      int64_t max_bytes);
int oracle_vcec_range(const void *img, int elem, int d, const int64_t *n, int64_t m, int64_t q0_lo, int64_t q0_hi,
                      int64_t *vcec);
int oracle_vcec3(const void *img, int elem, const int64_t *n, int64_t m, int64_t q0_lo, int64_t q0_hi,
                 int64_t *vcec, int nthreads);

static uint64_t state = 12345;
static uint32_t next_u32(void) {
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (uint32_t)(state >> 33);
}

int main(void) {
    const int64_t shapes[][4] = {{7, 1, 1, 1}, {5, 6, 1, 1}, {4, 5, 3, 1}, {1, 1, 1, 1}, {3, 2, 4, 2}, {9, 3, 8, 1}};
    const int dims[] = {1, 2, 3, 1, 4, 3};
    const int64_t m = 11;
    int fails = 0;
    for (int s = 0; s < 6; ++s) {
        const int d = dims[s];
        int64_t total = 1;
        for (int k = 0; k < d; ++k) total *= shapes[s][k];
        uint16_t *img = malloc((size_t)total * sizeof *img);
        int64_t *a = calloc((size_t)m, sizeof *a), *b = calloc((size_t)m, sizeof *b);
        for (int64_t i = 0; i < total; ++i) img[i] = (uint16_t)(next_u32() % m);
        for (int threads = 1; threads <= 4; threads += 3) {
            if (oracle_curve(img, 2, d, shapes[s], m, a, threads, 1 << 20) || a[m - 1] != 1) ++fails;
            if (oracle_curve_max(img, 2, d, shapes[s], m, a, threads, 1 << 20) || a[m - 1] != 1) ++fails;
            if (d <= 3 && oracle_curve_dual(img, 2, d, shapes[s], m, a, threads, 1 << 20)) ++fails;
            if (oracle_vcec(img, 2, d, shapes[s], m, a, threads, 1 << 20)) ++fails;
            if (d == 3) {
                memset(b, 0, (size_t)m * sizeof *b);
                if (oracle_vcec3(img, 2, shapes[s], m, 0, 2 * shapes[s][0] + 1, b, threads)) ++fails;
                for (int64_t t = 0; t < m; ++t) fails += a[t] != b[t];
                memset(a, 0, (size_t)m * sizeof *a);
                memset(b, 0, (size_t)m * sizeof *b);
                if (oracle_vcec_range(img, 2, 3, shapes[s], m, 1, 4, a)) ++fails;
                if (oracle_vcec3(img, 2, shapes[s], m, 1, 4, b, threads)) ++fails;
                for (int64_t t = 0; t < m; ++t) fails += a[t] != b[t];
            }
        }
        img[0] = (uint16_t)m;  /* out of range: rejected, nothing written out of bounds */
        if (oracle_curve(img, 2, d, shapes[s], m, a, 2, 1 << 20) != -2) ++fails;
        free(img);
        free(a);
        free(b);
    }
    printf("oracle sanitizer driver: %d failures\n", fails);
    return fails != 0;
}
