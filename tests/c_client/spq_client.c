/*
 * A plain C client of the library: no Python, no torch, host arrays only.
 * Reads a graph and query pairs from a binary file, builds the index with
 * spq_build_index_host (Algorithm 1), answers the pairs with
 * spq_query_batch_host, again with spq_query_batch_host_static (Algorithm
 * 2), and a third time through the library's server (spq_server_*, the
 * pairs submitted as requests of up to 700 pairs), and writes the three
 * answer arrays.
 *
 * Input file (int32 little endian): n, m, k, q, then eu[m], ev[m], w[m],
 * part[n], v1[q], v2[q].  Output file: out_host[q], out_static[q],
 * out_served[q].
 * Exit status 0 on success; a status code and spq_last_error() on stderr
 * otherwise.
 */
#include <stdio.h>
#include <stdlib.h>

#include "spq.h"

static int32_t* take(FILE* f, size_t count) {
  int32_t* p = (int32_t*)malloc(sizeof(int32_t) * (count ? count : 1));
  if (p && fread(p, sizeof(int32_t), count, f) != count) {
    free(p);
    return NULL;
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[4];
  if (fread(hdr, sizeof(int32_t), 4, f) != 4) return 2;
  const int32_t n = hdr[0], m = hdr[1], k = hdr[2], q = hdr[3];
  int32_t *eu = take(f, m), *ev = take(f, m), *w = take(f, m), *part = take(f, n);
  int32_t *v1 = take(f, q), *v2 = take(f, q);
  fclose(f);
  if (!eu || !ev || !w || !part || !v1 || !v2) return 2;
  spq_index* idx = NULL;
  spq_status st = spq_build_index_host(n, m, eu, ev, w, part, k, NULL, &idx);
  if (st != SPQ_OK) {
    fprintf(stderr, "build: %d %s\n", (int)st, spq_last_error());
    return 1;
  }
  int32_t* out = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)q);
  st = spq_query_batch_host(idx, q, v1, v2, out);
  if (st == SPQ_OK) st = spq_query_batch_host_static(idx, q, v1, v2, out + q, NULL);
  if (st == SPQ_OK) {
    spq_server* srv = NULL;
    st = spq_server_create(idx, 2, 1024, 1 << 16, &srv);
    const int32_t per = 700, nreq = (q + per - 1) / per;
    int64_t* tickets = (int64_t*)malloc(sizeof(int64_t) * (nreq ? nreq : 1));
    for (int32_t r = 0; r < nreq && st == SPQ_OK; r++) {
      const int32_t lo = r * per, cnt = q - lo < per ? q - lo : per;
      st = spq_server_submit(srv, cnt, v1 + lo, v2 + lo, out + 2 * (size_t)q + lo, &tickets[r]);
    }
    for (int32_t r = 0; r < nreq && st == SPQ_OK; r++) {
      int32_t done = 0;
      double lat = 0;
      st = spq_server_poll(srv, tickets[r], 1, &done, &lat);
      if (st == SPQ_OK && !done) st = SPQ_EDEVICE;
    }
    int64_t launches = 0, pairs = 0;
    if (st == SPQ_OK && spq_server_stats(srv, &launches, &pairs) == SPQ_OK)
      printf("served: %lld pairs in %lld launches\n", (long long)pairs, (long long)launches);
    spq_server_destroy(srv);
    free(tickets);
  }
  if (st != SPQ_OK) {
    fprintf(stderr, "query: %d %s\n", (int)st, spq_last_error());
    spq_free_index(idx);
    return 1;
  }
  spq_stats s;
  if (spq_index_stats(idx, &s) == SPQ_OK)
    printf("n=%d k=%d v_bg=%d bg_method=%d\n", s.n, s.k, s.v_bg, s.bg_method);
  spq_free_index(idx);
  f = fopen(argv[2], "wb");
  if (!f || fwrite(out, sizeof(int32_t), 3 * (size_t)q, f) != 3 * (size_t)q) return 2;
  fclose(f);
  free(out);
  free(eu); free(ev); free(w); free(part); free(v1); free(v2);
  return 0;
}
