/* Drives the CPU oracle's entry points on small inputs under the
 * sanitizers: a put/get program with every op kind, the collectives, the
 * reductions of every type, GUPS and the witness replay.  Checks a few
 * closed forms; prints "ok" and exits 0 when all hold. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint8_t op, scope, aux, flags;
    int32_t issuer, target;
    uint32_t result_idx;
    uint64_t src, dst, nbytes, value, cond, reserved;
} desc_t;

int orc_run_program(uint8_t *heap, int npes, uint64_t stride, const desc_t *d, uint64_t n, uint64_t *res,
                    uint64_t nres, int check, char *err, int errlen);
int orc_broadcast(uint8_t *heap, int npes, uint64_t stride, int start, int st, int size, uint64_t dst, uint64_t src,
                  uint64_t n, int root);
int orc_fcollect(uint8_t *heap, int npes, uint64_t stride, int start, int st, int size, uint64_t dst, uint64_t src,
                 uint64_t n);
int orc_alltoall(uint8_t *heap, int npes, uint64_t stride, int start, int st, int size, uint64_t dst, uint64_t src,
                 uint64_t n);
int orc_reduce(uint8_t *heap, int npes, uint64_t stride, int start, int st, int size, int dt, int rop, uint64_t dst,
               uint64_t src, uint64_t nreduce, const uint64_t *only, uint64_t nonly, void *out);
int orc_gups(int64_t *table, uint64_t nwords, const uint64_t *idx, const uint64_t *val, const uint8_t *is_add,
             uint64_t n, uint64_t *fetched);
int64_t orc_witness_check(const uint64_t *addr, const uint8_t *kind, const uint64_t *val, const uint64_t *fetched,
                          uint64_t nupd, const uint64_t *init, const uint64_t *final, uint64_t nwords, uint64_t budget);

static int failures;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); ++failures; } } while (0)

int main(void)
{
    enum { P = 5, S = 4096 };
    uint8_t *heap = malloc((size_t)P * S);
    for (int i = 0; i < P * S; ++i) heap[i] = (uint8_t)(i * 7 + 3);
    /* put, get, signal-put, every AMO kind, fence, quiet, barriers */
    desc_t d[16];
    memset(d, 0, sizeof d);
    int k = 0;
    d[k++] = (desc_t){1, 0, 0, 0, 0, 1, 0xFFFFFFFFu, 0, 1024, 100, 0, 0, 0};        /* put 0 -> 1 */
    d[k++] = (desc_t){2, 0, 0, 0, 2, 3, 0xFFFFFFFFu, 200, 1500, 77, 0, 0, 0};       /* get 2 <- 3 */
    d[k++] = (desc_t){13, 0, 0, 0, 0, 0, 0xFFFFFFFFu, 0, 0, 0, 0, 0, 0};            /* fence */
    d[k++] = (desc_t){3, 0, 0, 0, 4, 0, 0xFFFFFFFFu, 300, 2000, 64, 9, 3000, 0};    /* signal-put, SET */
    for (int p = 0; p < P; ++p) d[k++] = (desc_t){15, 0, 0, 0, p, p, 0xFFFFFFFFu, 0, 0, 0, 0, 0, 0};
    d[k++] = (desc_t){4, 0, 0, 0, 1, 2, 0, 3008, 0, 8, 5, 0, 0};                     /* fetch_add */
    d[k++] = (desc_t){5, 0, 0, 0, 1, 2, 1, 3016, 0, 8, 0xFF, 0, 0};                  /* fetch_xor */
    d[k++] = (desc_t){6, 0, 0, 0, 1, 2, 2, 3024, 0, 8, 42, 0, 0};                    /* compare_swap */
    d[k++] = (desc_t){14, 0, 0, 0, 1, 1, 0xFFFFFFFFu, 0, 0, 0, 0, 0, 0};             /* quiet */
    uint64_t res[3] = {0, 0, 0};
    char err[256];
    uint8_t *before = malloc((size_t)P * S);
    memcpy(before, heap, (size_t)P * S);
    CHECK(orc_run_program(heap, P, S, d, (uint64_t)k, res, 3, 1, err, 256) == 0);
    CHECK(memcmp(heap + 1 * S + 1024, before + 0 * S + 0, 100) == 0);
    CHECK(memcmp(heap + 2 * S + 1500, before + 3 * S + 200, 77) == 0);
    uint64_t sig;
    memcpy(&sig, heap + 0 * S + 3000, 8);
    CHECK(sig == 9);
    uint64_t w0;
    memcpy(&w0, before + 2 * S + 3008, 8);
    CHECK(res[0] == w0);
    /* collectives */
    CHECK(orc_broadcast(heap, P, S, 0, 1, P, 2048, 0, 300, 2) == 0);
    for (int p = 0; p < P; ++p) CHECK(memcmp(heap + p * S + 2048, heap + 2 * S, 300) == 0);
    CHECK(orc_fcollect(heap, P, S, 0, 1, P, 1024, 0, 100) == 0);
    CHECK(memcmp(heap + 4 * S + 1024 + 300, heap + 3 * S, 100) == 0);
    memcpy(before, heap, (size_t)P * S);
    CHECK(orc_alltoall(heap, P, S, 0, 1, P, 2048, 0, 64) == 0);
    CHECK(orc_alltoall(heap, P, S, 0, 1, P, 0, 2048, 64) == 0);
    for (int p = 0; p < P; ++p) CHECK(memcmp(heap + p * S, before + p * S, 64 * P) == 0);   /* involution */
    /* reductions: every type and op, strided team, sampled outputs */
    for (int dt = 0; dt < 3; ++dt)
        for (int rop = 0; rop < 2; ++rop) {
            CHECK(orc_reduce(heap, P, S, 0, 1, P, dt, rop, 3072, 2560, 60, NULL, 0, NULL) == 0);
            CHECK(orc_reduce(heap, P, S, 1, 2, 2, dt, rop, 3072, 2560, 60, NULL, 0, NULL) == 0);
            uint64_t only[3] = {0, 7, 59};
            uint8_t out[24];
            CHECK(orc_reduce(heap, P, S, 0, 1, P, dt, rop, 3072, 2560, 60, only, 3, out) == 0);
        }
    CHECK(orc_reduce(heap, P, S, 0, 1, P, 0, 0, 3072, 2560, 1000, NULL, 0, NULL) != 0);   /* out of range */
    /* GUPS and the witness replay of its fetched values */
    enum { N = 4000, T = 256 };
    int64_t *table = calloc(T, 8);
    uint64_t *idx = malloc(N * 8), *val = malloc(N * 8), *fet = malloc(N * 8), *init = calloc(T, 8);
    uint8_t *add = malloc(N), *kind = malloc(N);
    uint64_t s = 1;
    for (int u = 0; u < N; ++u) {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        idx[u] = (s >> 33) % T;
        val[u] = s;
        add[u] = (uint8_t)((s >> 20) % 5 == 0);
        kind[u] = add[u] ? 0 : 1;
    }
    CHECK(orc_gups(table, T, idx, val, add, N, fet) == 0);
    CHECK(orc_witness_check(idx, kind, val, fet, N, init, (const uint64_t *)table, T, 1u << 20) == 0);
    fet[17] ^= 1;
    CHECK(orc_witness_check(idx, kind, val, fet, N, init, (const uint64_t *)table, T, 1u << 20) >= 1);
    free(table); free(idx); free(val); free(fet); free(init); free(add); free(kind);
    free(heap);
    free(before);
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
