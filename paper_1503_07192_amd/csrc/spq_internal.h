// Internal declarations shared by the kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spq {

typedef uint32_t u32;

enum : u32 { ERR_PART = 1u, ERR_VERTEX = 2u, ERR_WEIGHT = 4u };

// Component tables are padded to a multiple of this side.
constexpr int COMP_TILE = 64;
// Components with more vertices are closed by the multi-workgroup blocked
// rounds (padded to 128) instead of one workgroup each.
constexpr int BIG_COMP = 1024;

struct PartArgs {
  int32_t n, k;
  int64_t m;
  const int32_t *eu, *ev, *w, *part;
  int32_t* cnt;               // [k] vertices per component
  int32_t* nb;                // [k] boundary vertices per component
  uint8_t* flag;              // [n] boundary flag
  unsigned long long* sumc;   // [k] weight of the edges inside each component
  unsigned long long* total;  // [1] weight of all edges
  u32* err;                   // [1] ERR_* bits
  const int32_t* off;         // [k+1] first vertex of each component
  const int32_t* bgoff;       // [k+1] first BG id of each component
  int32_t* fill;              // [k] scratch counters (zeroed)
  u32* members;               // [n] scratch
  int32_t *comp, *local;      // [n]
  int32_t *bgcomp, *bglocal;  // [V]
  int32_t* bgvert;            // [V] vertex of each BG id
  const int64_t* moff;        // [k] first element of each APSP(C)
  const int32_t* P;           // [k] padded side of each APSP(C)
  const int32_t *grp, *gbg0;  // [k] group of each component, [groups] its first BG id
  const int32_t* gV;          // [groups] BG vertices of each group
  const int64_t* gT;          // [groups] first element of the group's band in the blocked store
  u32* vrec;                  // [VREC_WORDS n] per-vertex query records
};
// Per-vertex query record (48 bytes):
//   0 1  first element of the vertex's APSP(C) row    2 component   3 local index
//   4    first BG id of the group                     5 |B(C)|      6 group
//   7    first BG id of the component inside its group
//   8    BG vertices of the group   9 unused   10 11 first element of the group's band
constexpr int VREC_WORDS = 12;

struct CompArgs {
  int32_t k;
  int64_t m;
  const int32_t *eu, *ev, *w, *comp, *local, *P;
  const int64_t* moff;
  u32* M;
};

struct BgArgs {
  int32_t V;
  int64_t Vp, m;
  const int32_t *eu, *ev, *w, *comp, *local, *bgoff, *nb, *bgcomp, *bglocal, *P;
  const int64_t* moff;
  const u32* M;
  u32* BG;
};

struct QueryArgs {
  int64_t q;
  const int32_t *v1, *v2;
  int32_t* out;
  int32_t n;
  const u32* vrec;
  const u32* M;
  const u32* H;  // blocked BG store (both methods)
  int32_t share_comps;  // > 0: only sources v1 in components [0, share_comps)
};

// Two-level BG (hier.hip).
struct HierArgs {
  int32_t V, ngroups, Vgp, m2pmax, V2, kc;
  int32_t pivot;  // rows per pivot block of the dense closures (128 or 256)
  hipStream_t side = nullptr;    // BG2 closure lookahead: side stream (default priority)
  hipEvent_t* sync = nullptr;    // and its two events; null: no lookahead
  int64_t m, V2p;
  const int32_t *eu, *ev, *w, *comp, *local, *bgoff, *nb, *bgcomp, *bglocal, *P;
  const int64_t* moff;
  const u32* M;
  const int32_t *grp, *gbg0, *gV;  // [k], [ngroups], [ngroups]
  int32_t *bgrow, *bgnb, *bggrp;   // [V]
  u32* Mg;                         // ngroups x Vgp x Vgp
  uint8_t* flag2;                  // [V]
  int32_t *b2list, *b2rank, *m2;   // ngroups x Vgp, [V], [ngroups]
  const int32_t* b2off;            // [ngroups+1]
  u32 *R, *XT, *BG2, *H;
  // the composition's positions (ngroups x Vrp, see hier.hip; NULL: local
  // indices, R and XT of leading dimension Vgp, every column in the second
  // product)
  int32_t* pos = nullptr;
  int32_t Vrp = 0;
  // BG2 as the first product reads it: dense (d2pstride = 0, leading
  // dimension V2p), or one column panel per group (share: S2p x m2pmax,
  // leading dimension d2ld = m2pmax, panels d2pstride apart)
  int64_t d2ld = 0, d2pstride = 0;
  const int64_t* pairbase;         // ngroups x ngroups
  // share mode: rows of BG only from the first share_groups groups
  int32_t share_groups, S2;        // groups, level-2 sources (ids 0 .. S2-1)
  int64_t S2p;                     // S2 rounded up to 128
  u32* DT;                         // Bellman-Ford distances (V2p + 128 rows x S2p)
  int4* xe;                        // directed cross edges
  int32_t* xcount;
  const int2* plist;               // composition: group pairs (S1, S2), see PAIR_SWAP
  const u32* D2t = nullptr;        // D2 transposed (rows: level-2 ids; the share's DT)
  int64_t d2tld = 0;               //   its leading dimension
  int32_t npairs, chunk;           //   their count, pairs per launch (XT slots)
  hipEvent_t* evt;                 // NULL, or 2 per composition launch (k_mp_y)
  // exactness certificate fused into the composition (NULL: off)
  const int32_t* bglabel;
  u32 *cert_bad, *cert_mbg;
};
// The share's Bellman-Ford blocks: runs of consecutive groups, nblk of them
// (block t = groups [bfirst[t], bfirst[t+1]), gblk[group] = its block;
// multi: some block holds more than one group); boff[nblk+1] first level-2
// id of each, bsize[nblk] level-2 vertices of each; A: nblk x bpmax x bpmax
// (BG2 induced on each block, closed).
// A pair of the level-2 composition whose y carries PAIR_SWAP is computed
// through the other boundary: (x, y & ~PAIR_SWAP) = (S2, S1) for the output
// block (S1, S2), so the large product runs over B2(S1) instead of B2(S2);
// its first product reads the D2 block transposed (D2t).
constexpr int32_t PAIR_SWAP = 0x40000000;
struct ShareBlocks {
  int32_t nblk, bpmax;
  bool multi;
  const int32_t *bfirst, *gblk, *boff, *bsize;
  u32* A;
};
hipError_t launch_share_prepare(const HierArgs& a, const ShareBlocks& b, hipStream_t s);
// The blocks' boundary B3: level-2 vertices with a G edge to another block,
// the only rows a cross edge lowers.  Lists hold local indices into a
// block's rows (bpmax slots per block): b3list the B3 rows, nb3list the
// others, both ascending; b3rank[level-2 id] = index in b3list (-1: not B3);
// m3 / n3 their counts.  A3: nblk x b3pmax x b3pmax, the closed block matrix
// on B3 x B3; Aout: nblk x b3pmax x n3pmax, on B3 (rows) x the other rows.
struct ShareB3 {
  int32_t b3pmax, n3pmax;
  const int32_t *m3, *n3, *b3list, *nb3list, *b3rank;
  u32 *A3, *Aout;
};
// flags from the cross edges (after launch_share_prepare), then the lists;
// flag3 / flagn: V2 bytes, nrank: V2 words of scratch
hipError_t launch_share_b3_lists(const HierArgs& a, const ShareBlocks& b, uint8_t* flag3,
                                 uint8_t* flagn, int32_t* b3list, int32_t* nb3list, int32_t* b3rank,
                                 int32_t* nrank, int32_t* m3, int32_t* n3, hipStream_t s);
// A3 and Aout gathered from the closed block matrices
hipError_t launch_share_b3_gather(const ShareBlocks& b, const ShareB3& c, hipStream_t s);
// After the rounds: rows outside B3 from the settled B3 rows,
//   DT[v] = min(DT[v], min over b in B3(T) of A_T[v][b] + DT[b])
hipError_t launch_share_final(const HierArgs& a, const ShareBlocks& b, const ShareB3& c,
                              hipStream_t s);
// One Bellman-Ford round of the share, on the B3 rows of every block.  dirty
// flags: per block, ntc = S2p / 128 column tiles then one "any" word; cnt /
// list: per (block, tile) the number of B3 rows lowered since the last intra
// step (BF_ALL_ROWS: all) and their indices in b3list (b3pmax slots each);
// stamp: V2p x ntc round stamps.
constexpr int32_t BF_ALL_ROWS = 0x7fffffff;
constexpr int BF_LDS_TILES = 2048;  // column tiles a cross-edge workgroup tracks in LDS
struct BfRound {
  const u32* dirty;
  u32* dirty_next;
  const int32_t* cnt;
  const int32_t* list;
  int32_t* cnt_next;
  int32_t* list_next;
  u32* stamp;
  u32 round;
};
hipError_t launch_share_round(const HierArgs& a, const ShareBlocks& b, const ShareB3& c, int32_t nxe,
                              const BfRound& r, hipStream_t s);
hipError_t launch_share_compose(const HierArgs& a, const u32* DT, hipStream_t s);
hipError_t launch_hier_level1(const HierArgs& a, hipStream_t s);
// Flat method: per-BG-vertex layout terms, then the closed BG matrix (Vp x Vp)
// copied into the blocked store of a single group.
hipError_t launch_flat_store(int32_t V, int64_t Vp, const u32* BG, const int32_t* bgcomp,
                             const int32_t* bgoff, const int32_t* nb, const int32_t* grp,
                             const int32_t* gbg0, int32_t* bgrow, int32_t* bgnb, int32_t* bggrp,
                             const int32_t* bglocal, u32* H, hipStream_t s);
// level 2 in three steps: R_S and the unclosed BG2 matrix; its closure by
// flat Floyd-Warshall (or by level 3 below); the composition into H
hipError_t launch_hier_level2_prep(const HierArgs& a, hipStream_t s);
hipError_t launch_hier_level2_close(const HierArgs& a, hipStream_t s);
hipError_t launch_hier_level2_compose(const HierArgs& a, hipStream_t s);

// Level 3: the closure of BG2 by the same construction on super-groups of
// gpt consecutive groups (hier.hip).
struct L3Args {
  int32_t nT, gpt, V3gp, V3, m3pmax, kc;
  int32_t pivot;  // rows per pivot block of the dense closures
  hipStream_t side = nullptr;    // BG3 closure lookahead (as for BG2)
  hipEvent_t* sync = nullptr;
  int64_t m, V2p, V3p;
  const int32_t *eu, *ev, *w, *comp, *local, *bgoff, *grp;
  const int32_t *b2off, *b2rank;       // level-2 ids
  u32* BG2;                            // V2p x V2p, unclosed in, closed (upper block triangle) out
  const int32_t *tbase, *tsize;        // [nT]: first BG2 id, BG2 vertices of each super-group
  u32* M3;                             // nT x V3gp x V3gp
  uint8_t* flag3;                      // [V2]
  int32_t *b3list, *b3rank, *m3;       // nT x V3gp, [V2], [nT]
  const int32_t* b3off;                // [nT+1]
  u32 *R3, *BG3;                       // nT x m3pmax x V3rp, V3p x V3p
  u32* XT3;                            // chunk x m3pmax x V3rp
  // the super-groups' positions (nT x V3rp, as the groups' at level 2;
  // NULL: local indices, V3rp = V3gp)
  int32_t* pos3 = nullptr;
  int32_t V3rp = 0;
  const int2* plist;                   // super-group pairs T1 <= T2
  int32_t npairs, chunk;               //   their count, pairs per launch
};
// super-group matrices, their closure, the level-3 boundary (m3)
hipError_t launch_level3_a(const L3Args& a, hipStream_t s);
// BG3 and its closure, then d_BG2 for super-group pairs T1 <= T2 into BG2
hipError_t launch_level3_b(const L3Args& a, hipStream_t s);
// the two products of the level-3 composition alone (pairs, XT3, R3, M3, BG3 ->
// BG2), a.chunk pairs per launch
hipError_t launch_level3_compose(const L3Args& a, hipStream_t s);
// the intra-group product of one Bellman-Ford round of the share, on its own
// The two Bellman-Ford products on caller buffers (test hooks): k_bf_intra3
// with group g owning rows own[g*lstride ..] of C and A[g] kp x kp, every
// tile dirty; k_bf_final with K rows own[g*lstride ..], output rows
// out[g*lstride ..] and Aout[g] kp x np.  zero: ngroups zeros (row offsets).
hipError_t launch_bf_rows(int32_t ngroups, int32_t lstride, int32_t kp, int64_t ldc,
                          const int32_t* nk, const int32_t* zero, const int32_t* own, const u32* A,
                          u32* C, const u32* dirty, const int32_t* rcnt, const int32_t* rlist,
                          hipStream_t s);
hipError_t launch_bf_gather(int32_t ngroups, int32_t lstride, int32_t kp, int32_t np, int64_t ldc,
                            const int32_t* nk, const int32_t* nout, const int32_t* zero,
                            const int32_t* own, const int32_t* out, const u32* Aout, u32* C,
                            hipStream_t s);
hipError_t launch_hier_row(const HierArgs& a, int32_t x, u32* out, hipStream_t s);

// Exactness certificate (range.hip).
struct CertArgs {
  bool bg_checked;  // BG entries already checked (fused into the two-level store)
  int32_t V, ngroups, Vgp;
  int64_t Vp, comp_elems;
  const u32 *M, *BG, *H;
  const int32_t *bgvert, *label, *gV, *gbg0, *bgrow, *bgnb, *bglocal;
  const int64_t* pairbase;
  int32_t* bglabel;
  u32 *bad, *mc, *mbg;
};
hipError_t launch_cc_init(int32_t n, int32_t* label, hipStream_t s);
hipError_t launch_cc_round(int64_t m, const int32_t* eu, const int32_t* ev, int32_t n, int32_t* label,
                           u32* changed, hipStream_t s);
hipError_t launch_certificate(const CertArgs& a, hipStream_t s);
hipError_t launch_bg_label(int32_t V, const int32_t* bgvert, const int32_t* label, int32_t* bglabel,
                           hipStream_t s);

hipError_t launch_partition_scan(const PartArgs& a, hipStream_t s);
hipError_t launch_renumber(const PartArgs& a, hipStream_t s);
// Edge validation and weight sums only (a.part may be the renumbered comp[]).
hipError_t launch_edges_scan(const PartArgs& a, hipStream_t s);
hipError_t launch_components(const CompArgs& a, hipStream_t s);
hipError_t launch_comp_fw(int32_t count, const int32_t* order, const int32_t* P, const int64_t* moff,
                          u32* M, hipStream_t s);
hipError_t launch_bg_assembly(const BgArgs& a, hipStream_t s);
// ev: NULL, or two events per round recorded around its interior-tile
// launch(es); kc: K chunk of the interior-tile kernel, 16 or 32 (0 = default);
// pivot: rows per pivot block, the tile (or 0) or twice the tile (see fw.hip)
hipError_t launch_dense_fw(u32* A, int64_t ld, int tile, int nt, hipStream_t s, hipEvent_t* ev,
                           int kc = 0, int pivot = 0);
// `batch` matrices of the same shape, gstride elements apart
hipError_t launch_dense_fw_batch(u32* A, int64_t ld, int tile, int nt, int batch, int64_t gstride,
                                 hipStream_t s, hipEvent_t* ev, int kc = 0, int pivot = 0);
// Same closure with a lookahead over two streams (side: created by the caller,
// default priority; sync: two events), or three with p1 (part 1 of every
// round beside part 2; sync: three events).
hipError_t launch_dense_fw_lookahead(u32* A, int64_t ld, int tile, int nt, hipStream_t s,
                                     hipStream_t side, hipEvent_t* sync, hipEvent_t* ev, int kc,
                                     int pivot = 0, hipStream_t p1 = nullptr);
// the lookahead closure of `batch` matrices, gstride elements apart
hipError_t launch_dense_fw_batch_lookahead(u32* A, int64_t ld, int tile, int nt, int batch,
                                           int64_t gstride, hipStream_t s, hipStream_t side,
                                           hipEvent_t* sync, hipEvent_t* ev, int kc, int pivot);
// rounds of a single-matrix closure (pivot blocks)
int fw_rounds_count(int nt, int tile, int pivot);
// relaxations executed by launch_dense_fw (diagonal, panel and upper-triangle
// interior tiles of every round); *inner (optional) = the interior part
double dense_fw_exec_relax(int64_t nt, int tile, int pivot = 0, double* inner = nullptr);
hipError_t launch_query(const QueryArgs& a, hipStream_t s);
// VALU rate probes (probe.hip): kind 0 v_add_u32, 1 v_min3_u32, 2 the
// relaxation loop on LDS operands; out: blocks * 256 words
hipError_t launch_valu_probe(int kind, int blocks, int iters, u32* out, hipStream_t s);
// Adjacency of G (both directions, self-loops dropped) as rowptr[n+1] and
// (neighbour, edge index) pairs; deg[n] zeroed scratch.
hipError_t launch_adjacency(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                            unsigned long long* deg, int64_t* rowptr, int2* adj, hipStream_t s);
// One shortest path per pair by a walk on the adjacency (kernels.hip).
hipError_t launch_paths(const QueryArgs& a, int32_t max_len, const int64_t* rowptr, const int2* adj,
                        const int32_t* wts, int32_t* paths, int32_t* lens, hipStream_t s);
// Sets this thread's spq_last_error message and returns s (api.hip).
int set_error(int s, const char* msg);

}  // namespace spq
