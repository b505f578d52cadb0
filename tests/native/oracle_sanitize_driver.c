/* Runs every entry point of the CPU oracle on small tie-heavy integer-grid
 * inputs, for a build under AddressSanitizer and UndefinedBehaviorSanitizer
 * (the CPU test suite compiles and runs it).  Checks that the interval-tree
 * matcher (sequential and threaded), brute force and, for d = 1, the sweep
 * return the same pairs; exits non-zero on any difference. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_itm(const float*, const float*, uint32_t, const float*, const float*, uint32_t,
               uint32_t, int, int, uint64_t**, uint64_t*);
int oracle_brute(const float*, const float*, uint32_t, const float*, const float*, uint32_t,
                 uint32_t, int, uint64_t**, uint64_t*);
int oracle_sbm_1d(const float*, const float*, uint32_t, const float*, const float*, uint32_t,
                  uint64_t**, uint64_t*);
int oracle_itm_1d_visits(const float*, const float*, uint32_t, const float*, const float*,
                         uint32_t, uint64_t*, uint32_t*, uint32_t*);
void oracle_free(void*);

static uint64_t rng_state = 88172645463325252ull;
static uint32_t next_u32(void) { /* xorshift64 */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 32);
}

static void draw(float* lo, float* hi, uint32_t count, uint32_t d) {
    for (uint32_t i = 0; i < count * d; ++i) {
        int a = (int)(next_u32() % 10) - 2;
        lo[i] = (float)a;
        hi[i] = (float)(a + (int)(next_u32() % 3));
        if (a == 0 && next_u32() % 8 == 0) lo[i] = -0.0f;
    }
}

static int same(const uint64_t* a, uint64_t na, const uint64_t* b, uint64_t nb) {
    return na == nb && (na == 0 || memcmp(a, b, na * sizeof(uint64_t)) == 0);
}

int main(void) {
    int bad = 0;
    for (int round = 0; round < 24; ++round) {
        uint32_t d = 1 + (uint32_t)round % 3;
        uint32_t n = next_u32() % 150, m = next_u32() % 150;
        float* s_lo = malloc(sizeof(float) * (n * d + 1));
        float* s_hi = malloc(sizeof(float) * (n * d + 1));
        float* u_lo = malloc(sizeof(float) * (m * d + 1));
        float* u_hi = malloc(sizeof(float) * (m * d + 1));
        draw(u_lo, u_hi, m, d);
        draw(s_lo, s_hi, n, d);
        uint64_t *k1 = NULL, *k2 = NULL, *k3 = NULL, *k4 = NULL;
        uint64_t c1 = 0, c2 = 0, c3 = 0, c4 = 0;
        bad |= oracle_itm(s_lo, s_hi, n, u_lo, u_hi, m, d, 1, 0, &k1, &c1) != 0;
        bad |= oracle_itm(s_lo, s_hi, n, u_lo, u_hi, m, d, 3, 0, &k2, &c2) != 0;
        bad |= oracle_brute(s_lo, s_hi, n, u_lo, u_hi, m, d, 0, &k3, &c3) != 0;
        bad |= !same(k1, c1, k3, c3) || !same(k2, c2, k3, c3);
        if (d == 1) {
            bad |= oracle_sbm_1d(s_lo, s_hi, n, u_lo, u_hi, m, &k4, &c4) != 0;
            bad |= !same(k4, c4, k3, c3);
            uint64_t* visits = malloc(sizeof(uint64_t) * (m + 1));
            uint32_t* hits = malloc(sizeof(uint32_t) * (m + 1));
            uint32_t H = 0;
            bad |= oracle_itm_1d_visits(s_lo, s_hi, n, u_lo, u_hi, m, visits, hits, &H) != 0;
            uint64_t tot = 0;
            for (uint32_t j = 0; j < m; ++j) tot += hits[j];
            bad |= tot != c3;
            free(visits);
            free(hits);
        }
        oracle_free(k1); oracle_free(k2); oracle_free(k3); oracle_free(k4);
        free(s_lo); free(s_hi); free(u_lo); free(u_hi);
    }
    /* invalid input is rejected, not read past */
    float lo[2] = {1.0f, 2.0f}, hi[2] = {0.5f, 3.0f};
    uint64_t* k = NULL;
    uint64_t c = 0;
    bad |= oracle_itm(lo, hi, 2, lo, lo, 2, 1, 1, 0, &k, &c) == 0;
    printf(bad ? "oracle sanitize driver: MISMATCH\n" : "oracle sanitize driver: ok\n");
    return bad;
}
