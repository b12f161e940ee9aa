/*
 * CPU oracle for shortest-path queries on a partitioned graph.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code with the HIP path.
 *
 * Everything is int64 with O_INF = INT64_MAX meaning "no path", so no
 * distance of an int32-weighted graph can overflow here.
 *
 *   oracle_dijkstra   textbook binary-heap Dijkstra on an undirected graph
 *                     (Section 1: O(m log n) single-source distances), one
 *                     independent run per requested source.
 *   oracle_fw         textbook Floyd-Warshall on a dense distance matrix
 *                     initialised to wt / infinity (Section 4, first
 *                     paragraph), the k loop outermost.
 *   oracle_query_alg2 the query algorithm (Algorithm 2) evaluated in the
 *                     paper's order: for each b2 of B(C2) the best b1 of
 *                     B(C1); then the best b2; then the C1 = C2 correction.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_INF INT64_MAX

static int64_t sat_add(int64_t a, int64_t b) {
  if (a == O_INF || b == O_INF) return O_INF;
  return a + b;
}

/* ------------------------------------------------------------ Dijkstra -- */
typedef struct {
  int32_t n;
  const int64_t* rowptr; /* CSR of the undirected graph, both directions */
  const int32_t* adj;
  const int64_t* wgt;
  const int32_t* src;
  int64_t nsrc;
  int64_t* out; /* nsrc x n */
  int64_t next; /* shared work counter */
  pthread_mutex_t lock;
} dj_job;

typedef struct { int64_t d; int32_t v; } heap_item;

static void heap_push(heap_item* h, int64_t* len, heap_item x) {
  int64_t i = (*len)++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= x.d) break;
    h[i] = h[p];
    i = p;
  }
  h[i] = x;
}

static heap_item heap_pop(heap_item* h, int64_t* len) {
  heap_item top = h[0], last = h[--(*len)];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= *len) break;
    if (c + 1 < *len && h[c + 1].d < h[c].d) c++;
    if (h[c].d >= last.d) break;
    h[i] = h[c];
    i = c;
  }
  if (*len > 0) h[i] = last;
  return top;
}

static void dijkstra_one(const dj_job* J, int32_t s, int64_t* dist, heap_item* heap) {
  int32_t n = J->n;
  for (int32_t v = 0; v < n; v++) dist[v] = O_INF;
  int64_t len = 0;
  dist[s] = 0;
  heap_item first = {0, s};
  heap_push(heap, &len, first);
  while (len > 0) {
    heap_item it = heap_pop(heap, &len);
    if (it.d != dist[it.v]) continue; /* stale entry */
    for (int64_t e = J->rowptr[it.v]; e < J->rowptr[it.v + 1]; e++) {
      int32_t u = J->adj[e];
      int64_t nd = it.d + J->wgt[e];
      if (nd < dist[u]) {
        dist[u] = nd;
        heap_item x = {nd, u};
        heap_push(heap, &len, x);
      }
    }
  }
}

static void* dj_worker(void* arg) {
  dj_job* J = (dj_job*)arg;
  int64_t hcap = J->rowptr[J->n] + 1;
  heap_item* heap = (heap_item*)malloc(sizeof(heap_item) * (size_t)hcap);
  if (!heap) return (void*)1;
  for (;;) {
    pthread_mutex_lock(&J->lock);
    int64_t i = J->next++;
    pthread_mutex_unlock(&J->lock);
    if (i >= J->nsrc) break;
    dijkstra_one(J, J->src[i], J->out + i * (int64_t)J->n, heap);
  }
  free(heap);
  return NULL;
}

/* Distances from each src[i] to every vertex: out[i*n + v].  Edges are
 * undirected; self-loops and parallel edges are allowed.  Returns 0, or -1 on
 * a bad argument or allocation failure. */
int oracle_dijkstra(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                    const int32_t* w, int64_t nsrc, const int32_t* src,
                    int64_t* out, int32_t nthreads) {
  if (n < 0 || m < 0 || nsrc < 0) return -1;
  for (int64_t e = 0; e < m; e++)
    if (eu[e] < 0 || eu[e] >= n || ev[e] < 0 || ev[e] >= n || w[e] < 0) return -1;
  for (int64_t i = 0; i < nsrc; i++)
    if (src[i] < 0 || src[i] >= n) return -1;
  int64_t* rowptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  int64_t* wgt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!rowptr || !adj || !wgt || !fill) return -1;
  for (int64_t e = 0; e < m; e++) {
    rowptr[eu[e] + 1]++;
    rowptr[ev[e] + 1]++;
  }
  for (int32_t v = 0; v < n; v++) rowptr[v + 1] += rowptr[v];
  memcpy(fill, rowptr, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t e = 0; e < m; e++) {
    adj[fill[eu[e]]] = ev[e];
    wgt[fill[eu[e]]++] = w[e];
    adj[fill[ev[e]]] = eu[e];
    wgt[fill[ev[e]]++] = w[e];
  }
  free(fill);
  dj_job J;
  J.n = n; J.rowptr = rowptr; J.adj = adj; J.wgt = wgt;
  J.src = src; J.nsrc = nsrc; J.out = out; J.next = 0;
  pthread_mutex_init(&J.lock, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  int rc = 0;
  for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, dj_worker, &J);
  for (int t = 0; t < nthreads; t++) {
    void* r = NULL;
    pthread_join(th[t], &r);
    if (r) rc = -1;
  }
  pthread_mutex_destroy(&J.lock);
  free(rowptr); free(adj); free(wgt);
  return rc;
}

/* ------------------------------------------------------ Floyd-Warshall -- */
/* In place on an N x N row-major matrix that holds 0 on the diagonal, the
 * edge weight where an edge exists and O_INF elsewhere. */
void oracle_fw(int32_t N, int64_t* d) {
  for (int32_t k = 0; k < N; k++)
    for (int32_t i = 0; i < N; i++) {
      int64_t dik = d[(int64_t)i * N + k];
      if (dik == O_INF) continue;
      for (int32_t j = 0; j < N; j++) {
        int64_t c = sat_add(dik, d[(int64_t)k * N + j]);
        if (c < d[(int64_t)i * N + j]) d[(int64_t)i * N + j] = c;
      }
    }
}

/* Floyd-Warshall on many independent matrices: matrix c has size[c] rows
 * and starts at element off[c]. */
typedef struct {
  int32_t count; const int32_t* size; const int64_t* off; int64_t* data;
  int64_t next; pthread_mutex_t lock;
} fw_job;

static void* fw_worker(void* arg) {
  fw_job* J = (fw_job*)arg;
  for (;;) {
    pthread_mutex_lock(&J->lock);
    int64_t i = J->next++;
    pthread_mutex_unlock(&J->lock);
    if (i >= J->count) break;
    oracle_fw(J->size[i], J->data + J->off[i]);
  }
  return NULL;
}

void oracle_fw_many(int32_t count, const int32_t* size, const int64_t* off,
                    int64_t* data, int32_t nthreads) {
  fw_job J;
  J.count = count; J.size = size; J.off = off; J.data = data; J.next = 0;
  pthread_mutex_init(&J.lock, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, fw_worker, &J);
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&J.lock);
}

/* ------------------------------------------------------ Algorithm 2 ------ */
/* Tables in the oracle's own layout:
 *   comp[v], pos[v]      component of v and v's index inside it
 *   csize[c], moff[c]    APSP(C) is csize[c] x csize[c] at apsp + moff[c]
 *   bstart[c..c+1]       boundary vertices of c are blocal[bstart[c]..bstart[c+1])
 *                        (indices inside c); the BG id of the i-th one is bstart[c]+i
 *   dbg                  V x V distances in BG
 * out[i] = dist(v1[i], v2[i]), O_INF if none. */
void oracle_query_alg2(int64_t q, const int32_t* v1, const int32_t* v2,
                       const int32_t* comp, const int32_t* pos,
                       const int32_t* csize, const int64_t* moff, const int64_t* apsp,
                       const int32_t* bstart, const int32_t* blocal,
                       int32_t V, const int64_t* dbg, int64_t* out) {
  int64_t* t = NULL;
  int32_t tcap = 0;
  for (int64_t i = 0; i < q; i++) {
    int32_t C1 = comp[v1[i]], C2 = comp[v2[i]];
    int32_t p1 = pos[v1[i]], p2 = pos[v2[i]];
    const int64_t* A1 = apsp + moff[C1];
    const int64_t* A2 = apsp + moff[C2];
    int32_t n1 = csize[C1], n2 = csize[C2];
    int32_t nb2 = bstart[C2 + 1] - bstart[C2];
    if (nb2 > tcap) { free(t); tcap = nb2; t = (int64_t*)malloc(sizeof(int64_t) * (size_t)tcap); }
    /* first stage: dist(v1, b2) through the best b1 */
    for (int32_t j = 0; j < nb2; j++) {
      int32_t g2 = bstart[C2] + j;
      t[j] = O_INF;
      for (int32_t a = bstart[C1]; a < bstart[C1 + 1]; a++) {
        int64_t d1 = A1[(int64_t)p1 * n1 + blocal[a]];      /* dist_C1(v1, b1) */
        int64_t c = sat_add(d1, dbg[(int64_t)a * V + g2]);  /* + dist_BG(b1, b2) */
        if (c < t[j]) t[j] = c;
      }
    }
    /* the paper moves a column of APSP(C2) between nodes here; one memory needs nothing */
    /* second stage: the best b2 */
    int64_t r = O_INF;
    for (int32_t j = 0; j < nb2; j++) {
      int64_t d2 = A2[(int64_t)blocal[bstart[C2] + j] * n2 + p2]; /* dist_C2(b2, v2) */
      int64_t c = sat_add(t[j], d2);
      if (c < r) r = c;
    }
    /* same component: the path may stay inside C1 */
    if (C1 == C2) {
      int64_t d = A1[(int64_t)p1 * n1 + p2];
      if (d < r) r = d;
    }
    out[i] = r;
  }
  free(t);
}

/* ------------------------------------------------------ min-plus product -- */
/* C = A (x) B over (min, +): C[i][j] = min over k of A[i][k] + B[k][j].
 * This is how distance tables compose through a separating vertex set: a
 * shortest path from i to j that meets the set splits at a vertex k of it
 * into an i-k part and a k-j part (the two stages of Algorithm 2, and the
 * same composition one level up in the two-level BG).  A is n x K, B is
 * K x p, C is n x p, all row-major; O_INF means no path, and with K = 0 every
 * entry of C is O_INF. */
void oracle_minplus(int32_t n, int32_t K, int32_t p, const int64_t* A, const int64_t* B,
                    int64_t* C) {
  for (int32_t i = 0; i < n; i++)
    for (int32_t j = 0; j < p; j++) {
      int64_t best = O_INF;
      for (int32_t k = 0; k < K; k++) {
        int64_t c = sat_add(A[(int64_t)i * K + k], B[(int64_t)k * p + j]);
        if (c < best) best = c;
      }
      C[(int64_t)i * p + j] = best;
    }
}
