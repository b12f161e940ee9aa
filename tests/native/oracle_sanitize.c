/*
 * Drives every entry point of oracle/oracle.c on random small graphs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer: any
 * out-of-bounds access, leak, signed overflow or misaligned access aborts
 * the run.  It also checks that the entry points agree with each other
 * (Dijkstra = Floyd-Warshall, min-plus squaring reaches the same distances,
 * Algorithm 2 with one component = Floyd-Warshall), so the run is a test and
 * not only a load.  Exit status 0 = clean.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define O_INF INT64_MAX

int oracle_dijkstra(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev, const int32_t* w,
                    int64_t nsrc, const int32_t* src, int64_t* out, int32_t nthreads);
void oracle_fw(int32_t N, int64_t* d);
void oracle_fw_many(int32_t count, const int32_t* size, const int64_t* off, int64_t* data,
                    int32_t nthreads);
void oracle_minplus(int32_t n, int32_t K, int32_t p, const int64_t* A, const int64_t* B, int64_t* C);
void oracle_query_alg2(int64_t q, const int32_t* v1, const int32_t* v2, const int32_t* comp,
                       const int32_t* pos, const int32_t* csize, const int64_t* moff,
                       const int64_t* apsp, const int32_t* bstart, const int32_t* blocal, int32_t V,
                       const int64_t* dbg, int64_t* out);

static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(uint32_t k) {
  rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
  return (uint32_t)(rs % k);
}

int main(void) {
  for (int trial = 0; trial < 300; trial++) {
    const int32_t n = 1 + (int32_t)rnd(12);
    const int64_t m = rnd(30);
    int32_t* eu = malloc(sizeof(int32_t) * (m + 1));
    int32_t* ev = malloc(sizeof(int32_t) * (m + 1));
    int32_t* w = malloc(sizeof(int32_t) * (m + 1));
    for (int64_t e = 0; e < m; e++) {
      eu[e] = (int32_t)rnd(n); ev[e] = (int32_t)rnd(n); w[e] = (int32_t)rnd(50);
    }
    int32_t* src = malloc(sizeof(int32_t) * n);
    for (int32_t v = 0; v < n; v++) src[v] = v;
    int64_t* dj = malloc(sizeof(int64_t) * n * n);
    if (oracle_dijkstra(n, m, eu, ev, w, n, src, dj, 1 + trial % 3) != 0) return 2;
    /* Floyd-Warshall on the dense initial matrix, twice (single and many) */
    int64_t* d = malloc(sizeof(int64_t) * n * n);
    for (int64_t i = 0; i < (int64_t)n * n; i++) d[i] = O_INF;
    for (int32_t v = 0; v < n; v++) d[(int64_t)v * n + v] = 0;
    for (int64_t e = 0; e < m; e++) {
      if (eu[e] == ev[e]) continue;
      int64_t* a = d + (int64_t)eu[e] * n + ev[e];
      int64_t* b = d + (int64_t)ev[e] * n + eu[e];
      if (w[e] < *a) *a = w[e];
      if (w[e] < *b) *b = w[e];
    }
    int64_t* d0 = malloc(sizeof(int64_t) * n * n);
    for (int64_t i = 0; i < (int64_t)n * n; i++) d0[i] = d[i];
    oracle_fw(n, d);
    int64_t off = 0;
    int32_t size = n;
    int64_t* d2 = malloc(sizeof(int64_t) * n * n);
    for (int64_t i = 0; i < (int64_t)n * n; i++) d2[i] = d0[i];
    oracle_fw_many(1, &size, &off, d2, 2);
    /* min-plus squaring of the initial matrix */
    int64_t* sq = malloc(sizeof(int64_t) * n * n);
    int64_t* t = malloc(sizeof(int64_t) * n * n);
    for (int64_t i = 0; i < (int64_t)n * n; i++) sq[i] = d0[i];
    for (int r = 0; r < 4; r++) {
      oracle_minplus(n, n, n, sq, sq, t);
      for (int64_t i = 0; i < (int64_t)n * n; i++) sq[i] = t[i];
    }
    /* Algorithm 2 with one component and an empty boundary: APSP(C) = FW on G */
    int32_t* comp = calloc(n, sizeof(int32_t));
    int64_t moff = 0;
    int32_t bstart[2] = {0, 0};
    int32_t blocal[1] = {0};
    int64_t dbg[1] = {0};
    int32_t* qa = malloc(sizeof(int32_t) * n * n);
    int32_t* qb = malloc(sizeof(int32_t) * n * n);
    for (int32_t i = 0; i < n; i++)
      for (int32_t j = 0; j < n; j++) { qa[i * n + j] = i; qb[i * n + j] = j; }
    int64_t* qo = malloc(sizeof(int64_t) * n * n);
    oracle_query_alg2((int64_t)n * n, qa, qb, comp, src, &size, &moff, d, bstart, blocal, 0, dbg, qo);
    for (int64_t i = 0; i < (int64_t)n * n; i++) {
      if (dj[i] != d[i] || d2[i] != d[i] || sq[i] != d[i] || qo[i] != d[i]) {
        fprintf(stderr, "trial %d: entry %lld disagrees\n", trial, (long long)i);
        return 1;
      }
    }
    free(eu); free(ev); free(w); free(src); free(dj); free(d); free(d0); free(d2); free(sq);
    free(t); free(comp); free(qa); free(qb); free(qo);
  }
  printf("oracle sanitizer run: 300 graphs clean\n");
  return 0;
}
