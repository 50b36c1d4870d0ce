/* Host-only run of the CPU oracle (oracle/oracle.c) and the multicore CPU
 * census (paper_1603_02655_amd/cpu/tc_cpu.cpp) on seeded random digraphs with
 * loops, repeated arcs and empty rows, built by tests/test_native_sanitizers.py
 * with ASan/UBSan: every census the oracle offers (single, multithreaded,
 * ranges, labelled) must agree with its own brute force and with the CPU
 * census.  Exit status 0 when all agree. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void *oracle_graph_new(int32_t n, int64_t m, const int32_t *src, const int32_t *dst);
void oracle_graph_free(void *h);
int oracle_census(void *h, uint64_t out[16]);
int oracle_census64(void *h, uint64_t out[64]);
int oracle_census_range(void *h, int32_t x0, int32_t x1, uint64_t out[16]);
int oracle_census_mt(void *h, int threads, uint64_t out[16]);
int oracle_brute(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int threads, uint64_t out[16]);
int oracle_table(uint8_t T[64]);
int tc_cpu_census(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t threads, uint64_t counts[16],
                  double *census_seconds);

static uint64_t rng_state = 0x16030265u;
static uint32_t next_u32(void) {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(rng_state >> 33);
}

int main(void) {
    int failures = 0;
    uint8_t T[64];
    if (oracle_table(T) != 0) return 1;
    for (int trial = 0; trial < 60; ++trial) {
        const int32_t n = (int32_t)(next_u32() % 70);
        const int64_t m = n ? (int64_t)(next_u32() % (uint32_t)(n * n / 2 + 1)) : 0;
        int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
        int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
        for (int64_t i = 0; i < m; ++i) {
            src[i] = (int32_t)(next_u32() % (uint32_t)n);
            dst[i] = (int32_t)(next_u32() % (uint32_t)n);   /* loops and repeats included */
        }
        uint64_t brute[16], one[16], mt[16], c64[64], fold[16] = {0}, parts[16] = {0}, cpu[16];
        if (oracle_brute(n, m, src, dst, 2, brute) != 0) ++failures;
        void *g = oracle_graph_new(n, m, src, dst);
        if (!g) { ++failures; free(src); free(dst); continue; }
        if (oracle_census(g, one) != 0 || memcmp(one, brute, sizeof(one)) != 0) ++failures;
        if (oracle_census_mt(g, 3, mt) < 0 || memcmp(mt, brute, sizeof(mt)) != 0) ++failures;
        if (oracle_census64(g, c64) != 0) ++failures;
        for (int c = 0; c < 64; ++c) fold[T[c]] += c64[c];
        if (memcmp(fold, brute, sizeof(fold)) != 0) ++failures;
        const int32_t cut = n ? (int32_t)(next_u32() % (uint32_t)n) : 0;
        uint64_t a[16], b[16];
        if (oracle_census_range(g, 0, cut, a) != 0 || oracle_census_range(g, cut, n, b) != 0) ++failures;
        for (int k = 1; k < 16; ++k) parts[k] = a[k] + b[k];
        parts[0] = brute[0];
        if (memcmp(parts, brute, sizeof(parts)) != 0) ++failures;
        if (tc_cpu_census(n, m, src, dst, 3, cpu, NULL) != 0 || memcmp(cpu, brute, sizeof(cpu)) != 0) ++failures;
        oracle_graph_free(g);
        free(src);
        free(dst);
    }
    /* a bad id is refused, not read */
    int32_t s1[1] = {0}, d1[1] = {5};
    if (oracle_graph_new(3, 1, s1, d1) != NULL) ++failures;
    uint64_t out[16];
    if (tc_cpu_census(3, 1, s1, d1, 1, out, NULL) != -1) ++failures;
    if (failures) {
        fprintf(stderr, "%d disagreement(s)\n", failures);
        return 1;
    }
    printf("oracle and CPU census agree with the brute force on 60 graphs\n");
    return 0;
}
