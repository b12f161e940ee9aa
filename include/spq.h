/*
 * spq.h - exact shortest-path distance queries on a partitioned planar graph,
 * computed on one AMD Instinct MI355X (gfx950).
 *
 * The data structure is the one of Chapuis & Djidjev, "Shortest-Path Queries
 * in Planar Graphs on GPU-Accelerated Architectures" (arXiv 1503.07192):
 *
 *   preprocessing (Algorithm 1)
 *     - the boundary: vertices with a neighbour in another component (Sec. 2);
 *       vertices are renumbered so that every component is contiguous and its
 *       boundary vertices come first (Sec. 4, Fig. 1);
 *     - APSP(C): all-pairs distances inside the subgraph induced by each
 *       component C (Phase 2);
 *     - BG: the boundary vertices, joined by the edges of G between them and,
 *       inside each component, by edges weighted with the APSP(C) distance;
 *       then all-pairs distances in BG (Phase 3; by Lemma 1 they equal the
 *       distances in G).
 *   query (Algorithm 2)
 *     dist(v1,v2) = min over b1 in B(C1), b2 in B(C2) of
 *                   dist_C1(v1,b1) + dist_BG(b1,b2) + dist_C2(b2,v2),
 *     and, when C1 = C2, also dist_C1(v1,v2).
 *
 * Arithmetic is exact int32.  SPQ_INF (2^31-1) means "no path".  Graphs are
 * undirected: the edge (u,v,w) may be walked both ways.  Every call returns a
 * status; nothing aborts or throws across this interface.  The library is
 * bound to the HIP device current at spq_build_index; call the other
 * functions with that device current.
 */
#ifndef SPQ_H
#define SPQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPQ_INF 2147483647
#define SPQ_BAD_PAIR (-1) /* query output for a vertex id outside [0, n) */

typedef enum {
  SPQ_OK = 0,
  SPQ_EINVAL = 1,  /* bad argument: id, weight, partition, empty component */
  SPQ_ENOMEM = 2,  /* device allocation failed */
  SPQ_EDEVICE = 3, /* a HIP call failed */
  SPQ_ERANGE = 4,  /* distances might not fit below SPQ_INF */
  SPQ_EBUSY = 5    /* the call's fixed device scratch is in use by an
                      overlapping call on the same device */
} spq_status;

typedef struct spq_index spq_index; /* opaque; owns all its device memory */

typedef struct {
  int32_t bg_tile;     /* tile of the BG Floyd-Warshall: 0 (default 128), 64, 128 */
  int32_t profile;     /* 1: time every launch of the dominant BG kernel with
                          HIP events (see spq_stats) */
  int32_t plain;       /* 1: one kernel launch per component for APSP(C)
                          instead of one launch for all (comparison path) */
  int32_t bg_method;   /* 0 auto (flat up to 32,768 BG vertices), 1 flat
                          Floyd-Warshall on all of BG, 2 two-level */
  int32_t group_comps; /* two-level: consecutive components per group
                          (0 = auto: about 4,096 BG vertices per group).  A
                          share build with 100 groups or more cuts a group
                          that is wider (in 128-tiles of BG vertices) than
                          the 99th percentile into halves of consecutive
                          components until it fits */
  int32_t share_comps; /* 0: the whole index.  s > 0: one GPU's share, the
                          paper's APSP_BG(C) for C in [0, s) only (Alg. 1,
                          Phase 3, done at the nodes owning those C): BG
                          rows from the share's boundary vertices to all of
                          BG; queries then need v1 in a share component.
                          Two-level method; the share is rounded up to whole
                          groups; needs the total edge weight below SPQ_INF */
  int32_t inner_kc;    /* K chunk of the Floyd-Warshall interior-tile kernel:
                          0 (default 16), 16 or 32 (see the autotuner) */
  int32_t flags;       /* SPQ_NO_LOOKAHEAD: Floyd-Warshall rounds on one
                          stream: without the overlap of the next round's
                          diagonal and panel work (flat BG; the two-level
                          group, super-group, BG2 and BG3 closures) and,
                          flat, of a round's two interior parts.
                          SPQ_GRAPH: the device work that depends on the
                          weights (Phase 2, BG assembly and closure) is
                          captured into HIP graphs, launched, and kept in the
                          index for spq_reweight_index; the index keeps
                          device copies of eu, ev, w (12 bytes per edge).
                          Not with share_comps or profile.
                          SPQ_PATHS: keep the graph's adjacency (20 bytes per
                          edge) for spq_query_paths */
  int32_t level3_groups; /* two-level: BG2 (the graph of the group boundaries)
                          is closed by flat Floyd-Warshall, or, above 16,384
                          BG2 vertices, by the same construction once more on
                          super-groups of consecutive groups (level 3).
                          0 auto (about 4,096 BG2 vertices per super-group),
                          -1 never, g > 0 always, g groups per super-group.
                          Share mode never builds BG2: there it sets the
                          blocks of its Bellman-Ford over BG2, g consecutive
                          groups per block (closed together, so a round
                          crosses a block instead of a group); 0 auto (about
                          1,024 level-2 vertices per block), -1 one group */
  int32_t group_bg;      /* two-level: > 0 forms the groups by size instead of
                          by count: consecutive components join a group while
                          it holds at most group_bg BG vertices (a larger
                          component gets a group of its own); overrides
                          group_comps */
  int32_t bg_pivot;      /* rows per pivot block of the flat BG Floyd-Warshall
                          (each round closes one block, then updates every
                          other tile through it): 1, 2 or 4 tiles (the last
                          blocks of a matrix may be smaller); the other
                          closures (large components, groups, BG2,
                          super-groups, BG3; 128-tiles) then use blocks of as
                          many tiles.  0 default: four tiles for the flat BG,
                          two (256 rows) for the other closures.  The answers
                          do not depend on it */
} spq_build_opts;

#define SPQ_NO_LOOKAHEAD 1
#define SPQ_GRAPH 2
#define SPQ_PATHS 4

typedef struct {
  int32_t n, k;            /* vertices, components */
  int64_t m;               /* edges as given */
  int32_t v_bg;            /* boundary vertices = BG vertices */
  int32_t v_bg_padded;     /* side of the padded Floyd-Warshall matrix: all of BG
                              (flat) or one group (two-level) */
  int32_t max_comp;        /* largest component */
  int32_t max_boundary;    /* largest |B(C)| */
  int64_t comp_bytes;      /* bytes of all APSP(C) tables (padded) */
  int64_t bg_bytes;        /* bytes of the blocked BG distance store the queries
                              read (flat: V_BG^2 * 4; the Floyd-Warshall matrix
                              is kept beside it) */
  double relax_comp;       /* sum over C of |C|^3: Floyd-Warshall relaxations, Phase 2 */
  double relax_bg;         /* v_bg^3: Floyd-Warshall relaxations in BG, Phase 3 */
  double relax_comp_exec;  /* relaxations the kernels execute for Phase 2 (padded
                              tiles; symmetric tiles computed once) */
  double relax_bg_exec;    /* same for BG */
  double relax_dominant;   /* executed by the launches of the dominant BG kernel:
                              interior tiles (flat) or the composition product
                              (two-level, share) */
  int64_t dominant_launches; /* number of those launches */
  float ms_dominant;       /* their summed device time (only with opts.profile) */
  int32_t bg_method;       /* 1 flat, 2 two-level */
  int32_t ngroups;         /* groups of the two-level method (1 when flat) */
  int32_t v_bg2;           /* level-2 boundary vertices (two-level) */
  int32_t share_comps;     /* share mode: components [0, share_comps) (0 = all) */
  int32_t share_groups;    /* share mode: groups holding them */
  int32_t bf_rounds;       /* share mode: Bellman-Ford rounds over blocks of groups */
  float ms_partition;      /* device time: boundary, renumbering (through the host plan) */
  float ms_components;     /* device time: APSP(C) initialisation + Floyd-Warshall */
  float ms_bg_assembly;    /* device time: BG matrix assembly */
  float ms_bg_apsp;        /* device time: the BG closure (flat rounds, or every
                              level of the two-level method).  With SPQ_GRAPH
                              the phases run as one graph: ms_components and
                              ms_bg_assembly are 0 and ms_bg_apsp covers
                              Phases 2 and 3 */
  int32_t graphs;          /* HIP graphs held for spq_reweight_index (0 without SPQ_GRAPH) */
  int32_t reweights;       /* successful spq_reweight_index calls */
  int64_t graph_nodes;     /* nodes (kernel launches, event waits) in those graphs */
  int32_t groups3;         /* level-3 super-groups (0: BG2 closed flat) */
  int32_t v_bg3;           /* level-3 boundary vertices */
  int32_t bf_block_groups; /* share mode: groups per Bellman-Ford block */
} spq_stats;

/*
 * Preprocessing, Algorithm 1.
 *   n, m          vertex and edge counts (n >= 1, m >= 0)
 *   eu, ev, w     DEVICE arrays of m int32: edge (eu[i], ev[i]) of weight w[i];
 *                 0 <= w < SPQ_INF; self-loops are ignored; parallel edges
 *                 keep the lightest
 *   part          DEVICE array of n int32 in [0, k): the component of each
 *                 vertex (the k-partition of Section 2); every component
 *                 must be non-empty
 *   opts          may be NULL
 *   stream        hipStream_t the work is queued on (NULL = default stream)
 *   out           receives the index; on error *out is NULL
 * The inputs are read during the call only and stay owned by the caller.
 * The call blocks until the partition sizes are known (one small device to
 * host copy), then queues the remaining work on `stream` and returns; the
 * index is usable by work queued later on the same stream.
 * BG distances are closed either by Floyd-Warshall on the whole BG matrix
 * (flat) or by the two-level method: BG split into groups of consecutive
 * components, each group closed, the graph of the group boundaries closed,
 * and the remaining distances composed as in Algorithm 2 one level up.  Both
 * give the same distances.  The distances are then kept in a blocked store
 * where each B(C1) x B(C2) block is one contiguous run (what a query reads).
 * Errors: SPQ_EINVAL (bad id, weight or part, empty component, k < 1, bad
 * option, more than 32,768 groups),
 * SPQ_ERANGE (a distance might not fit below SPQ_INF: when the total edge
 * weight reaches SPQ_INF the build proves its result instead of assuming it
 * (every component's weight below SPQ_INF, no BG distance lost between
 * connected vertices, no query sum reaching SPQ_INF) and fails if it cannot;
 * a share build needs the total below SPQ_INF), SPQ_ENOMEM, SPQ_EDEVICE.
 */
spq_status spq_build_index(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                           const int32_t* w, const int32_t* part, int32_t k,
                           const spq_build_opts* opts, void* stream, spq_index** out);

/*
 * Preprocessing (Algorithm 1) from HOST arrays, for callers without device
 * memory of their own: the same arguments, options and results as
 * spq_build_index, but eu, ev, w (m int32 each) and part (n int32) are host
 * arrays, caller-owned and read during the call only.  They are copied into
 * device memory of the library, the build runs on a stream of the library's
 * own, and the call returns when the index is complete (the staging copies
 * are freed by then).  Use the index on any stream afterwards.
 * Errors: as spq_build_index (SPQ_ENOMEM also for the staging copies).
 */
spq_status spq_build_index_host(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                                const int32_t* w, const int32_t* part, int32_t k,
                                const spq_build_opts* opts, spq_index** out);

/*
 * Queries, Algorithm 2: out[i] = dist(v1[i], v2[i]) for i < q.
 *   v1, v2, out   DEVICE arrays of q int32, owned by the caller
 *   stream        hipStream_t (NULL = default stream); the call is asynchronous
 * A pair with an id outside [0, n), or (share mode) with v1 outside the
 * share's components, yields SPQ_BAD_PAIR in its slot; other slots are
 * unaffected.  Read-only on the index: calls may run concurrently
 * on different streams.  Errors: SPQ_EINVAL (null index, q < 0), SPQ_ERANGE
 * (index invalidated by a failed spq_reweight_index), SPQ_EDEVICE.
 */
spq_status spq_query_batch(const spq_index* idx, int64_t q, const int32_t* v1,
                           const int32_t* v2, int32_t* out, void* stream);

/*
 * The same queries on HOST arrays (v1, v2, out: q int32 each, caller-owned),
 * for callers without device memory of their own: the pairs are staged in
 * device memory of the library (allocated per call), answered on a stream
 * of the library's own, and copied back; returns when out is filled.
 * Synchronous.  Errors: as spq_query_batch, plus SPQ_ENOMEM.
 */
spq_status spq_query_batch_host(const spq_index* idx, int64_t q, const int32_t* v1,
                                const int32_t* v2, int32_t* out);

/*
 * spq_query_batch_host without any allocation, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * allocation after set-up): the pairs and answers are staged in a fixed
 * device array of the library, 3 x SPQ_STATIC_PAIRS int32 (12 MiB) per
 * device, set up on the first call on each device and held until the
 * process ends.  The call allocates nothing (no hipMalloc, no stream).
 *   v1, v2, out   HOST arrays of q int32, caller-owned, q <= SPQ_STATIC_PAIRS
 *   stream        hipStream_t the copies and the query kernel are queued on
 *                 (NULL = default stream)
 * Returns when out is filled (synchronous on `stream`).  Every call on a
 * device shares that device's array: overlapping calls would race, so a
 * call made while another one holds the array returns SPQ_EBUSY (nothing
 * done).  Nothing in the array needs clearing: each call writes the pairs
 * and answers it reads.
 * Errors: as spq_query_batch, plus SPQ_EINVAL (q > SPQ_STATIC_PAIRS),
 * SPQ_EBUSY.
 */
#define SPQ_STATIC_PAIRS (1 << 20)
spq_status spq_query_batch_host_static(const spq_index* idx, int64_t q, const int32_t* v1,
                                       const int32_t* v2, int32_t* out, void* stream);

/*
 * New edge weights for an index built with SPQ_GRAPH: same graph (eu, ev in
 * the same order), same partition, so the boundary, the renumbering, the
 * group plan and every launch shape stay; Phases 2 and 3 are recomputed by
 * replaying the captured graphs on `stream`.
 *   w       DEVICE array of m int32 (m as built), 0 <= w < SPQ_INF; read
 *           during the call only
 *   stream  hipStream_t (NULL = default stream); the call validates w (one
 *           small device to host copy), queues the replay after the index's
 *           last build or reweight, and returns (with the exactness
 *           certificate, below, it waits for the replay)
 * Queries queued later on `stream` see the new distances; queries still
 * running on other streams must finish first (the caller orders them).
 * When the total weight reaches SPQ_INF the result is certified as in the
 * build (connected components are computed once, on first need).
 * Errors: SPQ_EINVAL (NULL index, index built without SPQ_GRAPH, bad weight;
 * the index is unchanged), SPQ_ERANGE (a component's weights reach SPQ_INF:
 * index unchanged; or the certificate fails after the replay: the index is
 * invalid and every later query or reweight on it returns SPQ_ERANGE),
 * SPQ_EDEVICE.
 */
spq_status spq_reweight_index(spq_index* idx, const int32_t* w, void* stream);

/*
 * Shortest paths (index built with SPQ_PATHS): for pair i, the vertices of one
 * shortest path from v1[i] to v2[i], found by walking back from v2[i] over
 * neighbours u with dist(v1, u) + w(u, c) = dist(v1, c), each distance an
 * Algorithm 2 query on the index (no extra table per distance).
 *   v1, v2     DEVICE arrays of q int32
 *   max_len    room per path (>= 1)
 *   paths      DEVICE array of q * max_len int32: path i in
 *              paths[i * max_len .. i * max_len + lens[i]), from v1[i] to v2[i]
 *   lens       DEVICE array of q int32: vertices on the path (>= 1; 1 when
 *              v1 = v2), 0 no path, -1 bad pair (id outside [0, n), or v1
 *              outside a share), -2 the walk needed more than max_len
 *              vertices, -3 it found no way off a plateau of zero-weight edges
 *              (it backs out of dead ends but remembers only the last 16; with
 *              positive weights it never backs out)
 * Where several shortest paths exist any one may be returned.  Asynchronous
 * on `stream`.  Errors: SPQ_EINVAL (NULL index or array, q < 0, max_len < 1,
 * index built without SPQ_PATHS), SPQ_ERANGE (invalidated index),
 * SPQ_EDEVICE.
 */
spq_status spq_query_paths(const spq_index* idx, int64_t q, const int32_t* v1, const int32_t* v2,
                           int32_t max_len, int32_t* paths, int32_t* lens, void* stream);

/*
 * Continuous-batching server on a built index.  Answering many queries at
 * once is the extension the paper names as future work (Section 5); every
 * launch runs Algorithm 2 (spq_query_batch) on a batch of pairs.
 *
 * Requests (HOST arrays of pairs) are queued in submission order.  A worker
 * thread of the server coalesces the requests at the head of the queue into
 * launches on `slots` HIP streams (at most slot_pairs pairs per launch) and
 * writes each request's answers into its own output array.  The buffers of a
 * launch (12 bytes per pair: v1, v2, answer) are taken from one device pool
 * and one pinned host pool of mem_bytes each, both allocated at creation; a
 * launch starts only when a slot is free and its buffers can be allocated in
 * the pools (first fit), and returns them when it completes.  A request is
 * cut into several launches only when the room left in a launch cannot hold
 * it whole.  The answers are those of spq_query_batch on the same pairs.
 *
 *   spq_server_create   slots in [1, 64], slot_pairs >= 1, mem_bytes in
 *                       [256 B, 64 GiB] (rounded down to 256 B); waits for
 *                       the index build.  The index must outlive the
 *                       server and must not be reweighted while it runs.
 *                       Errors: SPQ_EINVAL, SPQ_ENOMEM, SPQ_EDEVICE.
 *   spq_server_submit   queues q pairs (q >= 0; q = 0 completes at once);
 *                       v1, v2 and out stay owned by the caller and must stay
 *                       valid, and out unread, until the request completes.
 *                       *ticket identifies the request.  Thread-safe.
 *                       Errors: SPQ_EINVAL, or the server's first device
 *                       error once one happened (nothing queued).
 *   spq_server_poll     *done = 1 once every answer of the ticket's request is
 *                       in its out array (wait != 0 blocks until then); then
 *                       *latency_s (may be NULL) = completion time minus
 *                       submission time, and the ticket is released (a later
 *                       poll of it returns SPQ_EINVAL).  Thread-safe.
 *                       Errors: SPQ_EINVAL (unknown ticket), the server's
 *                       first device error for a request it did not finish.
 *   spq_server_stats    launches made and pairs launched so far (either
 *                       pointer may be NULL).
 *   spq_server_destroy  answers every request submitted so far, then stops
 *                       the worker and frees the pools; NULL is ok.
 * After a device error the server answers nothing more: requests not yet
 * complete report the error, and so does every later submission.
 */
typedef struct spq_server spq_server;
spq_status spq_server_create(const spq_index* idx, int32_t slots, int64_t slot_pairs,
                             int64_t mem_bytes, spq_server** out);
spq_status spq_server_submit(spq_server* srv, int64_t q, const int32_t* v1, const int32_t* v2,
                             int32_t* out, int64_t* ticket);
spq_status spq_server_poll(spq_server* srv, int64_t ticket, int32_t wait, int32_t* done,
                           double* latency_s);
spq_status spq_server_stats(spq_server* srv, int64_t* launches, int64_t* pairs);
void spq_server_destroy(spq_server* srv);

/* Sizes, work counts and per-phase device times (waits for the build). */
spq_status spq_index_stats(const spq_index* idx, spq_stats* st);

/*
 * The renumbering (Section 4, Fig. 1), copied to HOST arrays (any may be NULL):
 *   comp[n]    component of each vertex
 *   local[n]   index of the vertex inside its component; boundary vertices
 *              take 0 .. nb[c]-1 in ascending id order, then the interior
 *              vertices in ascending id order
 *   nb[k]      |B(C)|
 *   off[k+1]   first renumbered vertex of each component
 *   bgoff[k+1] first BG vertex of each component (BG id = bgoff[c] + local)
 * Synchronous.
 */
spq_status spq_index_layout(const spq_index* idx, int32_t* comp, int32_t* local,
                            int32_t* nb, int32_t* off, int32_t* bgoff);

/* APSP(C) of component c, |C| x |C| int32 row-major in the local order above,
 * copied to the HOST array out.  Synchronous. */
spq_status spq_index_component(const spq_index* idx, int32_t c, int32_t* out);

/* Rows [row0, row0+nrows) of the BG distance matrix (v_bg columns each),
 * copied to the HOST array out.  In share mode only rows of the share's
 * groups exist (SPQ_EINVAL otherwise).  Synchronous. */
spq_status spq_index_bg_rows(const spq_index* idx, int32_t row0, int32_t nrows,
                             int32_t* out);

/* Releases the index (waits for the device).  Its device memory goes to the
 * library's cache and is reused by later builds; NULL is ok. */
void spq_free_index(spq_index* idx);

/* Frees the device memory and destroys the streams cached from released
 * indexes (all devices). */
void spq_release_cached_memory(void);

/* Message of the last error on this thread ("" if none). */
const char* spq_last_error(void);

/*
 * Test hooks: the Floyd-Warshall kernels on caller-owned DEVICE buffers.
 * Inputs must be symmetric (undirected graphs), 0 on the diagonal, with
 * entries in [0, SPQ_INF]; they are closed in place to all-pairs distances.
 *
 * spq_fw_components: count matrices; matrix i has side size[i] (HOST array)
 *   and starts at element off[i] (HOST array) of `data`; its leading
 *   dimension is ld[i] (HOST array), a multiple of 64 with ld[i] >= size[i].
 *   Rows and columns in [size[i], ld[i]) must hold SPQ_INF off the diagonal
 *   and 0 on it.  One workgroup closes one whole matrix (the APSP(C) kernel).
 * spq_fw_dense: one v x v matrix with leading dimension ld (a multiple of
 *   tile, padded like above); blocked Floyd-Warshall in rounds over pivot
 *   blocks of `pivot` rows (the BG kernels).  tile is 64 or 128; pivot is 1,
 *   2 or 4 tiles (0: one tile); kc (K chunk of the interior kernel) is 0
 *   (default), 16 or 32.
 * spq_fw_components stages its size tables on the device and returns when
 * the work is done; spq_fw_dense is asynchronous on `stream`.
 * Errors: SPQ_EINVAL, SPQ_ENOMEM, SPQ_EDEVICE.
 */
/*
 * Measurement hook: issue rates of the VALU instructions the min-plus kernels
 * are built from, on the current device (8 workgroups of 256 lanes per CU,
 * timed with HIP events on `stream`; about 0.1 s; synchronous).
 *   out[0]  v_add_u32 lane-operations per second (independent chains)
 *   out[1]  v_min3_u32 lane-operations per second (independent chains)
 *   out[2]  relaxations per second of the kernels' inner loop on LDS
 *           operands (no global memory in the loop)
 *   out[3]  relaxations per second of the same relaxation instructions on
 *           operands in registers (no LDS reads): the instruction sequence
 *           alone
 * out holds 4 doubles.  A relaxation is one add and half a min3, so out[0]
 * and out[1] bound the relaxation peak.  Errors: SPQ_EINVAL (out NULL), SPQ_ENOMEM, SPQ_EDEVICE.
 */
spq_status spq_valu_rates(double* out, void* stream);

spq_status spq_fw_components(int32_t count, const int32_t* size, const int64_t* off,
                             const int32_t* ld, int32_t* data, void* stream);
spq_status spq_fw_dense(int32_t v, int32_t ld, int32_t tile, int32_t pivot, int32_t kc, int32_t* data,
                        void* stream);

/*
 * Test hook: the min-plus products of the two-level build's group-level
 * composition, on caller-owned DEVICE buffers, by the kernels the build uses.
 * The composition is Algorithm 2 applied one level up (Lemma 3 with groups of
 * components in place of components): a shortest path from vertex x of group
 * S1 to vertex y of group S2 leaves S1 through a boundary vertex a and enters
 * S2 through a boundary vertex b, so
 *   T(S1,S2)[x][y] = min over a < nk[S1], b < nk[S2] of
 *                    R[S1][a][x] + D[koff[S1]+a][koff[S2]+b] + R[S2][b][y],
 *   also min'd with M[S1][x][y] when S1 = S2,
 * with every sum clamped at SPQ_INF (exact: outputs are min(exact, SPQ_INF)).
 *   layout    SPQ_MP_BLOCKED: the first product into a scratch table, then
 *             the product stored in the query layout (the two-level kernels);
 *             SPQ_MP_DENSE: the same first product, then the product stored
 *             densely (the level-3 kernels)
 *   groups    G in [1, 4096]; nv[g] in [1, vp] vertices and nk[g] in [0, kp]
 *             boundary rows per group (HOST arrays of G);
 *             koff[g] = nk[0] + ... + nk[g-1], voff[g] likewise over nv
 *   vp, kp    positive multiples of 128, vp <= 32,768
 *   R         G x kp x vp int32: R[g][a][x] at R[(g*kp + a)*vp + x]
 *   D         rows and columns koff[G] at least, leading dimension ldd >=
 *             koff[G] (may be NULL when koff[G] = 0)
 *   Dt        D transposed, same leading dimension: read when assoc != 0
 *             (NULL otherwise)
 *   M         G x vp x vp int32: M[g][x][y] at M[(g*vp + x)*vp + y]
 *   pairs     HOST array of 2*npairs group ids (S1, S2), no pair twice
 *   assoc     0: every pair through B2(S2) (the first product over B2(S1));
 *             2: every pair with S1 != S2 through B2(S1) instead (the
 *             products' roles exchanged, the first one reading Dt, the tile
 *             stored transposed); 1: per pair whichever costs fewer executed
 *             relaxations, as a share build chooses (1 and 2 need
 *             SPQ_MP_BLOCKED).  The result does not depend on it.
 *   out       SPQ_MP_BLOCKED: pair p's nv[S1] x nv[S2] values start at element
 *             obase[p] = sum over earlier pairs q of nv[S1_q]*nv[S2_q]; each
 *             group is cut into consecutive runs ("components") of cb
 *             vertices (the last may be shorter) and (x, y) sits at
 *             r(x)*nv[S2] + n(x)*r(y) + l(x)*n(y) + l(y), where r(v) = v - v%cb
 *             is the run's first vertex, n(v) its length and l(v) = v%cb
 *             (ldo unused).
 *             SPQ_MP_DENSE: (x, y) at out[(voff[S1]+x)*ldo + voff[S2]+y],
 *             ldo >= voff[G] (cb unused).
 * Every entry of R, D and M, padding included, must be in [0, SPQ_INF]
 * (entries are not checked).  Reads R rows past nk[g] up to the next
 * multiple of 16 and every column of R and M, never multiplying them into
 * an output.  Synchronous on `stream`; scratch memory is the library's.
 * Errors: SPQ_EINVAL, SPQ_ENOMEM, SPQ_EDEVICE.
 */
#define SPQ_MP_BLOCKED 0
#define SPQ_MP_DENSE 1
spq_status spq_minplus_batched(int32_t layout, int32_t groups, const int32_t* nv, const int32_t* nk,
                               int32_t vp, int32_t kp, const int32_t* R, const int32_t* D,
                               const int32_t* Dt, int64_t ldd, const int32_t* M, int32_t npairs,
                               const int32_t* pairs, int32_t assoc, int32_t cb, int32_t* out,
                               int64_t ldo, void* stream);

/*
 * Test hook: the intra-block product of the share build's Bellman-Ford
 * rounds (BG rows of one GPU's share, Algorithm 1 Phase 3, computed over
 * blocks of the two-level method's groups), in place on a caller-owned
 * DEVICE table C.  Group g owns nk[g] rows of C: own_g[r] = own[koff[g] + r]
 * (koff as above; own NULL: own_g[r] = koff[g] + r).  For each of them and
 * every column j < ldc:
 *   C[own_g[r]][j] = min(C[own_g[r]][j],
 *                        min over listed k of A[g][r][k] + C[own_g[k]][j]).
 *   nk        HOST array of G (in [1, 65535]) row counts in [0, kp]
 *   kp        positive multiple of 128
 *   A         G x kp x kp int32, A[g][r][k] at A[(g*kp + r)*kp + k]; must be
 *             symmetric on [0, nk[g])^2 (the kernel reads column r as row r)
 *   C         int32 rows of ldc (a positive multiple of 128) entries, at
 *             least every row named by own_g
 *   cnt       HOST array of G: cnt[g] < 0 lists every row 0 .. nk[g]-1, else
 *             the next cnt[g] entries of `rows` (HOST, indices r < nk[g])
 *             are the listed rows of group g
 *   own       HOST array of koff[G] distinct rows of C, or NULL
 * Rows are updated in place while other workgroups read them as K, so the
 * result is the formula above for any schedule only when every value read
 * is no smaller than it: A[g] closed (its own all-pairs distances, 0 on the
 * diagonal) and every row that is not listed already satisfying
 * A[g][r][k] + C[own_g[k]][j] >= C[own_g[r]][j] (the state between two
 * rounds).  Entries in [0, SPQ_INF].  Synchronous on `stream`.
 * Errors: SPQ_EINVAL, SPQ_ENOMEM, SPQ_EDEVICE.
 */
spq_status spq_minplus_rows(int32_t groups, const int32_t* nk, int32_t kp, const int32_t* A,
                            int32_t* C, int64_t ldc, const int32_t* cnt, const int32_t* rows,
                            const int32_t* own, void* stream);

/*
 * Test hook: the last product of the share build's Bellman-Ford stage, which
 * fills the rows of a block that no cross edge reaches from its boundary
 * rows, in place on a caller-owned DEVICE table C.  Group g reads nk[g] rows
 * own_g[k] = own[koff[g] + k] and writes nout[g] rows out_g[i] =
 * out[ooff[g] + i] (koff, ooff: exclusive prefix sums of nk, nout); for
 * every column j < ldc:
 *   C[out_g[i]][j] = min(C[out_g[i]][j],
 *                        min over k < nk[g] of Aout[g][k][i] + C[own_g[k]][j]).
 *   nk, nout  HOST arrays of G (in [1, 65535]) counts in [0, kp], [0, np]
 *   kp, np    positive multiples of 128
 *   Aout      G x kp x np int32, Aout[g][k][i] at Aout[(g*kp + k)*np + i]
 *   C         int32 rows of ldc (a positive multiple of 128) entries
 *   own, out  HOST arrays of koff[G] and ooff[G] rows of C; no row may be
 *             both read (own) and written (out)
 * Entries in [0, SPQ_INF].  Synchronous on `stream`.
 * Errors: SPQ_EINVAL, SPQ_ENOMEM, SPQ_EDEVICE.
 */
spq_status spq_minplus_gather(int32_t groups, const int32_t* nk, const int32_t* nout, int32_t kp,
                              int32_t np, const int32_t* Aout, int32_t* C, int64_t ldc,
                              const int32_t* own, const int32_t* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SPQ_H */
