// Two-level all-pairs distances in BG.
//
// The preprocessing of Algorithm 1 applied once more, one level up: BG itself
// is partitioned into groups of consecutive components.  For a group S:
//   * BG_S = the subgraph of BG induced by S's boundary vertices (the clique
//     edges of S's components plus the G edges between them), closed by
//     Floyd-Warshall: d_S (a batch of equally sized matrices);
//   * B2(S) = vertices of BG_S with a BG edge leaving S (the boundary of the
//     group partition, Section 2's definition applied to BG).
// BG2 = the B2 vertices of all groups, joined by d_S between the B2 vertices
// of one group and by the G edges between groups; closed by Floyd-Warshall it
// holds d_BG between B2 vertices (Lemma 1 for the group partition).  Every
// other BG distance is Algorithm 2's formula at the group level (Lemma 3):
//   D(S1,S2)[x][y] = min over a in B2(S1), b in B2(S2) of
//                    d_S1(x,a) + d_BG2(a,b) + d_S2(b,y),
//   and when S1 = S2 also d_S1(x,y).
// It is evaluated as two min-plus products, XT = D2(S1,S2)^T (x) R_S1 and
// D = XT^T (x) R_S2, where R_S = rows B2(S) of d_S (by symmetry, the columns
// too).  Only S1 <= S2 is stored; a query swaps its endpoints otherwise.
//
// Storage of D(S1,S2) (V_S1 x V_S2 values at pairbase[S1][S2]): the rows of
// one component C1 of S1 form a band; inside it, the block of component C2 of
// S2 is nb(C1) x nb(C2) contiguous values, so a query reads one contiguous
// block.  Element (x, y) is at
//   rowoff(x) * V_S2 + nb(x) * rowoff(y) + loc(x) * nb(y) + loc(y)
// with rowoff = first BG id of the component inside its group, loc = index
// inside the component's boundary.
#include "spq_internal.h"
#include "tiles.h"

namespace spq {

// Group matrix init: 0 on the diagonal, the APSP(C) distance inside one
// component, INF elsewhere and on the padding.
__global__ void k_grp_init(int32_t Vgp, const int32_t* __restrict__ gbg0, const int32_t* __restrict__ gV,
                           const int32_t* __restrict__ bgcomp, const int32_t* __restrict__ bglocal,
                           const int32_t* __restrict__ bgoff, const int32_t* __restrict__ nb,
                           const int32_t* __restrict__ P, const int64_t* __restrict__ moff,
                           const u32* __restrict__ M, u32* __restrict__ Mg) {
  const int s = blockIdx.y;
  const int64_t p = blockIdx.x;
  u32* out = Mg + ((int64_t)s * Vgp + p) * Vgp;
  const int32_t g0 = gbg0[s];
  int64_t lo = 0, hi = 0;
  const u32* mrow = nullptr;
  if (p < gV[s]) {
    const int32_t x = g0 + (int32_t)p;
    const int32_t c = bgcomp[x];
    lo = bgoff[c] - g0;
    hi = lo + nb[c];
    mrow = M + moff[c] + (int64_t)bglocal[x] * P[c] - lo;
  }
  for (int64_t q0 = (int64_t)threadIdx.x * 4; q0 < Vgp; q0 += (int64_t)blockDim.x * 4) {
    u32 v[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int64_t q = q0 + t;
      v[t] = (q == p) ? 0u : (q >= lo && q < hi) ? mrow[q] : INF;
    }
    *reinterpret_cast<uint4*>(out + q0) = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

// G edges between boundary vertices of different components: inside a group
// they become entries of the group matrix; between groups they mark both ends
// as level-2 boundary vertices.
__global__ void k_grp_edges(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            const int32_t* __restrict__ w, const int32_t* __restrict__ comp,
                            const int32_t* __restrict__ local, const int32_t* __restrict__ bgoff,
                            const int32_t* __restrict__ grp, const int32_t* __restrict__ gbg0,
                            int32_t Vgp, u32* __restrict__ Mg, uint8_t* __restrict__ flag2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = eu[e], v = ev[e];
    const int32_t cu = comp[u], cv = comp[v];
    if (cu == cv) continue;
    const int32_t su = grp[cu], sv = grp[cv];
    const int32_t xu = bgoff[cu] + local[u], xv = bgoff[cv] + local[v];
    if (su == sv) {
      u32* base = Mg + (int64_t)su * Vgp * Vgp;
      const int64_t a = xu - gbg0[su], b = xv - gbg0[su];
      atomicMin(base + a * Vgp + b, (u32)w[e]);
      atomicMin(base + b * Vgp + a, (u32)w[e]);
    } else {
      flag2[xu] = 1;
      flag2[xv] = 1;
    }
  }
}

// One workgroup per group: lists the level-2 boundary vertices of the group in
// ascending order (b2list), their rank (b2rank, -1 if not one) and count.
__global__ __launch_bounds__(256) void k_b2_scan(const int32_t* __restrict__ gbg0,
                                                 const int32_t* __restrict__ gV,
                                                 const uint8_t* __restrict__ flag2, int32_t Vgp,
                                                 int32_t* __restrict__ b2list, int32_t* __restrict__ b2rank,
                                                 int32_t* __restrict__ m2) {
  __shared__ int32_t wsum[4];
  const int s = blockIdx.x;
  const int32_t g0 = gbg0[s], V = gV[s];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t base = 0;
  for (int32_t c0 = 0; c0 < V; c0 += 256) {
    const int32_t p = c0 + (int32_t)threadIdx.x;
    const bool f = p < V && flag2[g0 + p];
    const unsigned long long bal = __ballot(f);
    const int32_t before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    int32_t woff = 0, tot = 0;
    for (int i = 0; i < 4; i++) {
      if (i < wid) woff += wsum[i];
      tot += wsum[i];
    }
    if (p < V) {
      if (f) {
        const int32_t r = base + woff + before;
        b2list[(int64_t)s * Vgp + r] = p;
        b2rank[g0 + p] = r;
      } else {
        b2rank[g0 + p] = -1;
      }
    }
    base += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) m2[s] = base;
}

// R_S: rows B2(S) of d_S (m2pmax rows per group, INF rows past m2[S]).
__global__ void k_r_gather(int32_t Vgp, int32_t m2pmax, const int32_t* __restrict__ m2,
                           const int32_t* __restrict__ b2list, const u32* __restrict__ Mg,
                           u32* __restrict__ R) {
  const int s = blockIdx.y;
  const int32_t i = blockIdx.x;
  uint4* dst = reinterpret_cast<uint4*>(R + ((int64_t)s * m2pmax + i) * Vgp);
  const int32_t n4 = Vgp / 4;
  if (i < m2[s]) {
    const uint4* src =
        reinterpret_cast<const uint4*>(Mg + ((int64_t)s * Vgp + b2list[(int64_t)s * Vgp + i]) * Vgp);
    for (int32_t q = threadIdx.x; q < n4; q += blockDim.x) dst[q] = src[q];
  } else {
    for (int32_t q = threadIdx.x; q < n4; q += blockDim.x) dst[q] = make_uint4(INF, INF, INF, INF);
  }
}

// Positions of every group (one workgroup each; the layout is described with
// the composition below): B2 vertices, padding to a multiple of 4, the other
// vertices ascending (found by b2rank < 0), padding up to Vrp.
__global__ __launch_bounds__(256) void k_pos_build(const int32_t* __restrict__ gbg0,
                                                   const int32_t* __restrict__ gV,
                                                   const int32_t* __restrict__ b2rank,
                                                   const int32_t* __restrict__ b2list,
                                                   const int32_t* __restrict__ m2, int32_t Vgp,
                                                   int32_t Vrp, int32_t* __restrict__ pos) {
  __shared__ int32_t wsum[4];
  const int s = blockIdx.x;
  const int32_t g0 = gbg0[s], V = gV[s], k = m2[s], P2 = (k + 3) & ~3, W = P2 + V - k;
  int32_t* out = pos + (int64_t)s * Vrp;
  for (int32_t p = threadIdx.x; p < Vrp; p += 256) {
    if (p < k) out[p] = b2list[(int64_t)s * Vgp + p];
    else if (p < P2 || p >= W) out[p] = -1;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t base = 0;
  for (int32_t c0 = 0; c0 < V; c0 += 256) {
    const int32_t p = c0 + (int32_t)threadIdx.x;
    const bool f = p < V && b2rank[g0 + p] < 0;
    const unsigned long long bal = __ballot(f);
    const int32_t before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    int32_t woff = 0, tot = 0;
    for (int i = 0; i < 4; i++) {
      if (i < wid) woff += wsum[i];
      tot += wsum[i];
    }
    if (f) out[P2 + base + woff + before] = p;
    base += tot;
    __syncthreads();
  }
}

// R_S by position: R[S][r][p] = d_S(r-th B2 vertex, vertex at position p) for
// r < m2[S]; INF on the other rows and at padding positions.
__global__ void k_rpos_gather(int32_t Vgp, int32_t Vrp, int32_t m2pmax, const int32_t* __restrict__ m2,
                              const int32_t* __restrict__ b2list, const int32_t* __restrict__ pos,
                              const u32* __restrict__ Mg, u32* __restrict__ R) {
  const int s = blockIdx.y;
  const int32_t i = blockIdx.x;
  u32* dst = R + ((int64_t)s * m2pmax + i) * Vrp;
  const bool live = i < m2[s];
  const u32* src = Mg + ((int64_t)s * Vgp + (live ? b2list[(int64_t)s * Vgp + i] : 0)) * Vgp;
  const int32_t* ps = pos + (int64_t)s * Vrp;
  for (int32_t p = threadIdx.x; p < Vrp; p += blockDim.x) {
    const int32_t x = live ? ps[p] : -1;
    dst[p] = x >= 0 ? src[x] : INF;
  }
}

// BG2 matrix init: d_S between B2 vertices of one group, 0 on the diagonal,
// INF elsewhere and on the padding.
__global__ void k_bg2_init(int32_t V2, int64_t V2p, int32_t ngroups, const int32_t* __restrict__ b2off,
                           const int32_t* __restrict__ b2list, int32_t Vgp, const u32* __restrict__ Mg,
                           u32* __restrict__ BG2) {
  const int64_t i = blockIdx.x;
  u32* out = BG2 + i * V2p;
  int64_t lo = 0, hi = 0;
  const u32* prow = nullptr;
  const int32_t* list = nullptr;
  if (i < V2) {
    int32_t a = 0, b = ngroups - 1;  // group of B2 id i: largest s with b2off[s] <= i
    while (a < b) {
      const int32_t mid = (a + b + 1) >> 1;
      if (b2off[mid] <= i) a = mid; else b = mid - 1;
    }
    lo = b2off[a];
    hi = b2off[a + 1];
    list = b2list + (int64_t)a * Vgp;
    prow = Mg + ((int64_t)a * Vgp + list[i - lo]) * Vgp;
  }
  for (int64_t q0 = (int64_t)threadIdx.x * 4; q0 < V2p; q0 += (int64_t)blockDim.x * 4) {
    u32 v[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int64_t q = q0 + t;
      v[t] = (q == i) ? 0u : (q >= lo && q < hi) ? prow[list[q - lo]] : INF;
    }
    *reinterpret_cast<uint4*>(out + q0) = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

__global__ void k_bg2_edges(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            const int32_t* __restrict__ w, const int32_t* __restrict__ comp,
                            const int32_t* __restrict__ local, const int32_t* __restrict__ bgoff,
                            const int32_t* __restrict__ grp, const int32_t* __restrict__ b2off,
                            const int32_t* __restrict__ b2rank, int64_t V2p, u32* __restrict__ BG2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = eu[e], v = ev[e];
    const int32_t cu = comp[u], cv = comp[v];
    if (cu == cv) continue;
    const int32_t su = grp[cu], sv = grp[cv];
    if (su == sv) continue;
    const int64_t a = b2off[su] + b2rank[bgoff[cu] + local[u]];
    const int64_t b = b2off[sv] + b2rank[bgoff[cv] + local[v]];
    atomicMin(BG2 + a * V2p + b, (u32)w[e]);
    atomicMin(BG2 + b * V2p + a, (u32)w[e]);
  }
}

// Per BG vertex: first BG id of its component inside its group, and the
// component's boundary count (the layout terms of D(S1,S2)).
__global__ void k_hier_vmeta(int32_t V, const int32_t* __restrict__ bgcomp, const int32_t* __restrict__ bgoff,
                             const int32_t* __restrict__ nb, const int32_t* __restrict__ grp,
                             const int32_t* __restrict__ gbg0, int32_t* __restrict__ bgrow,
                             int32_t* __restrict__ bgnb, int32_t* __restrict__ bggrp) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= V) return;
  const int32_t c = bgcomp[x], s = grp[c];
  bgrow[x] = bgoff[c] - gbg0[s];
  bgnb[x] = nb[c];
  bggrp[x] = s;
}

// Flat method: row x of the closed BG matrix into the blocked store of one
// group (the layout above with S1 = S2 = the only group).
__global__ void k_flat_store(int32_t V, int64_t Vp, const u32* __restrict__ BG,
                             const int32_t* __restrict__ bgrow, const int32_t* __restrict__ bgnb,
                             const int32_t* __restrict__ bglocal, u32* __restrict__ H) {
  const int64_t x = blockIdx.x;
  const u32* row = BG + x * Vp;
  const int64_t rb = (int64_t)bgrow[x] * V, nbx = bgnb[x], locx = bglocal[x];
  for (int32_t y = threadIdx.x; y < V; y += blockDim.x)
    H[rb + nbx * bgrow[y] + locx * bgnb[y] + bglocal[y]] = row[y];
}

// ------------------------------------------------------- min-plus products --
// c (128 x 128 in registers) = min(c, min over k < K of At[k][i] + B[k][j]).
// Rows k of At and B are ldA / ldB apart; K is a multiple of 16 and is
// streamed through LDS 16 rows at a time (double buffered, next chunk
// prefetched into registers).  With MASKED, rows k >= kvalid and columns
// i >= avalid of At read as INF without touching memory, and rows k >= kvalid
// of B likewise.  Rows of c at or past rv are left unfinished (never
// stored by the caller).
template <bool MASKED>
__device__ __forceinline__ uint4 mp_load_a(const u32* At, int64_t ldA, int k, int col, int kvalid,
                                           int avalid) {
  if (!MASKED) return *reinterpret_cast<const uint4*>(At + (int64_t)k * ldA + col);
  if (k >= kvalid) return make_uint4(INF, INF, INF, INF);
  const u32* p = At + (int64_t)k * ldA + col;
  if (col + 3 < avalid) return *reinterpret_cast<const uint4*>(p);
  return make_uint4(col < avalid ? p[0] : INF, col + 1 < avalid ? p[1] : INF,
                    col + 2 < avalid ? p[2] : INF, INF);
}

template <bool MASKED>
__device__ __forceinline__ uint4 mp_load_b(const u32* B, int64_t ldB, int k, int col, int kvalid) {
  if (MASKED && k >= kvalid) return make_uint4(INF, INF, INF, INF);
  return *reinterpret_cast<const uint4*>(B + (int64_t)k * ldB + col);
}

// The relaxations of one LDS chunk for a thread's first NR rows (8 all, 4
// the first half of the tile, 0 none: the wave only stages chunks) and its
// first NC columns (8 all, 4 the first half).
template <int NR, int NC = 8>
__device__ __forceinline__ void mp_chunk(u32 (&c)[8][8], const u32* sA, const u32* sB, int K) {
  if (NR > 0) minplus_lds<128, NR, NC>(c, sA, sB, K);
}

// The rows a wave relaxes when only rows below rv of the tile are ever
// stored: a thread's rows are h*64 + ty*4 + a and a wave holds four
// consecutive ty (16 rows of each half), so a wave whose rows of the second
// half (or of both halves) all lie at or past rv skips them, and its VALU
// slots go to the other waves of its SIMD.  Every wave still stages its
// share of each chunk and meets every barrier.
__device__ __forceinline__ int wave_rows(int rv) {
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  return (rv >= 128 || 64 + 16 * w < rv) ? 8 : (16 * w < rv) ? 4 : 0;
}

template <bool MASKED, int NR, int NC>
__device__ __forceinline__ void mp_stream128_n(u32 (&c)[8][8], const u32* At, int64_t ldA, const u32* B,
                                               int64_t ldB, int K, int kvalid, int avalid, u32* sA,
                                               u32* sB) {
  constexpr int T = 128, KC = 16;
  const int nch = K / KC;
  if (nch <= 0) return;
  // two uint4 of each operand per thread per chunk: rows e/32, columns 4*(e%32)
  const int e0 = threadIdx.x, e1 = threadIdx.x + 256;
  const int r0 = e0 >> 5, c0 = (e0 & 31) * 4, r1 = e1 >> 5, c1 = (e1 & 31) * 4;
  uint4 pa0 = mp_load_a<MASKED>(At, ldA, r0, c0, kvalid, avalid);
  uint4 pa1 = mp_load_a<MASKED>(At, ldA, r1, c1, kvalid, avalid);
  uint4 pb0 = mp_load_b<MASKED>(B, ldB, r0, c0, kvalid);
  uint4 pb1 = mp_load_b<MASKED>(B, ldB, r1, c1, kvalid);
  reinterpret_cast<uint4*>(sA)[e0] = pa0;
  reinterpret_cast<uint4*>(sA)[e1] = pa1;
  reinterpret_cast<uint4*>(sB)[e0] = pb0;
  reinterpret_cast<uint4*>(sB)[e1] = pb1;
  __syncthreads();
  for (int ch = 0; ch < nch; ch++) {
    // the last iteration reloads its own chunk into the idle buffer (unused)
    const int kn = (ch + 1 < nch ? ch + 1 : ch) * KC;
    pa0 = mp_load_a<MASKED>(At, ldA, kn + r0, c0, kvalid, avalid);
    pa1 = mp_load_a<MASKED>(At, ldA, kn + r1, c1, kvalid, avalid);
    pb0 = mp_load_b<MASKED>(B, ldB, kn + r0, c0, kvalid);
    pb1 = mp_load_b<MASKED>(B, ldB, kn + r1, c1, kvalid);
    const int cur = (ch & 1) * KC * T, nxt = ((ch + 1) & 1) * KC * T;
    mp_chunk<NR, NC>(c, sA + cur, sB + cur, KC);
    reinterpret_cast<uint4*>(sA + nxt)[e0] = pa0;
    reinterpret_cast<uint4*>(sA + nxt)[e1] = pa1;
    reinterpret_cast<uint4*>(sB + nxt)[e0] = pb0;
    reinterpret_cast<uint4*>(sB + nxt)[e1] = pb1;
    __syncthreads();
  }
}

// Columns of c at or past cv are likewise left unfinished: when cv <= 64
// every thread relaxes only its columns of the tile's first half (a branch
// uniform over the workgroup).
template <bool MASKED>
__device__ __forceinline__ void mp_stream128(u32 (&c)[8][8], const u32* At, int64_t ldA, const u32* B,
                                             int64_t ldB, int K, int kvalid, int avalid, u32* sA,
                                             u32* sB, int rv = 128, int cv = 128) {
  const int nr = wave_rows(rv);
  if (nr == 0)
    mp_stream128_n<MASKED, 0, 8>(c, At, ldA, B, ldB, K, kvalid, avalid, sA, sB);
  else if (cv > 64) {
    if (nr == 8)
      mp_stream128_n<MASKED, 8, 8>(c, At, ldA, B, ldB, K, kvalid, avalid, sA, sB);
    else
      mp_stream128_n<MASKED, 4, 8>(c, At, ldA, B, ldB, K, kvalid, avalid, sA, sB);
  } else {
    if (nr == 8)
      mp_stream128_n<MASKED, 8, 4>(c, At, ldA, B, ldB, K, kvalid, avalid, sA, sB);
    else
      mp_stream128_n<MASKED, 4, 4>(c, At, ldA, B, ldB, K, kvalid, avalid, sA, sB);
  }
}

// c = min(c, min over k < cnt of At[rows[k]][i] + B[bmap[rows[k]]][j]): the K
// rows are gathered through the list `rows` (rows k themselves when it is
// null; cnt of them, streamed 16 at a time, rows past cnt read as INF without
// touching memory), and B's rows once more through bmap when it is not null.
template <int NR>
__device__ __forceinline__ void mp_stream128_rows_n(u32 (&c)[8][8], const u32* At, int64_t ldA,
                                                    const u32* B, int64_t ldB,
                                                    const int32_t* __restrict__ rows, int cnt,
                                                    u32* sA, u32* sB,
                                                    const int32_t* __restrict__ bmap) {
  constexpr int T = 128, KC = 16;
  const int nch = (cnt + KC - 1) / KC;
  if (nch <= 0) return;
  const int e0 = threadIdx.x, e1 = threadIdx.x + 256;
  const int r0 = e0 >> 5, c0 = (e0 & 31) * 4, r1 = e1 >> 5, c1 = (e1 & 31) * 4;
  const uint4 inf4 = make_uint4(INF, INF, INF, INF);
  auto lda = [&](int k, int col) -> uint4 {
    if (k >= cnt) return inf4;
    return *reinterpret_cast<const uint4*>(At + (int64_t)(rows ? rows[k] : k) * ldA + col);
  };
  auto ldb = [&](int k, int col) -> uint4 {
    if (k >= cnt) return inf4;
    const int32_t r = rows ? rows[k] : k;
    return *reinterpret_cast<const uint4*>(B + (int64_t)(bmap ? bmap[r] : r) * ldB + col);
  };
  uint4 pa0 = lda(r0, c0), pa1 = lda(r1, c1);
  uint4 pb0 = ldb(r0, c0), pb1 = ldb(r1, c1);
  reinterpret_cast<uint4*>(sA)[e0] = pa0;
  reinterpret_cast<uint4*>(sA)[e1] = pa1;
  reinterpret_cast<uint4*>(sB)[e0] = pb0;
  reinterpret_cast<uint4*>(sB)[e1] = pb1;
  __syncthreads();
  for (int ch = 0; ch < nch; ch++) {
    const int kn = (ch + 1 < nch ? ch + 1 : ch) * KC;
    pa0 = lda(kn + r0, c0);
    pa1 = lda(kn + r1, c1);
    pb0 = ldb(kn + r0, c0);
    pb1 = ldb(kn + r1, c1);
    const int cur = (ch & 1) * KC * T, nxt = ((ch + 1) & 1) * KC * T;
    mp_chunk<NR>(c, sA + cur, sB + cur, KC);
    reinterpret_cast<uint4*>(sA + nxt)[e0] = pa0;
    reinterpret_cast<uint4*>(sA + nxt)[e1] = pa1;
    reinterpret_cast<uint4*>(sB + nxt)[e0] = pb0;
    reinterpret_cast<uint4*>(sB + nxt)[e1] = pb1;
    __syncthreads();
  }
}

__device__ __forceinline__ void mp_stream128_rows(u32 (&c)[8][8], const u32* At, int64_t ldA,
                                                  const u32* B, int64_t ldB,
                                                  const int32_t* __restrict__ rows, int cnt,
                                                  u32* sA, u32* sB,
                                                  const int32_t* __restrict__ bmap = nullptr) {
  // every row: the gathered operands leave no registers for a second copy
  // of the loop (the kernels' last row tiles are a small share of them)
  mp_stream128_rows_n<8>(c, At, ldA, B, ldB, rows, cnt, sA, sB, bmap);
}

// The composition kernels fit in 128 VGPRs without spilling: four waves per
// SIMD (four workgroups per CU) instead of two or three.
#define SPQ_MP_ATTR __attribute__((amdgpu_waves_per_eu(4, 4)))

// c = min(c, the 128 x 128 tile at g), in the register layout of tile_load.
__device__ __forceinline__ void tile_min128(u32 (&c)[8][8], const u32* __restrict__ g, int64_t ld) {
  const int tx = tid_x(), ty = tid_y();
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int a = 0; a < 4; a++) {
      const u32* row = g + (int64_t)(h * 64 + ty * 4 + a) * ld + tx * 4;
#pragma unroll
      for (int h2 = 0; h2 < 2; h2++) {
        const uint4 v = *reinterpret_cast<const uint4*>(row + h2 * 64);
        u32* r = c[h * 4 + a] + h2 * 4;
        r[0] = min(r[0], v.x);
        r[1] = min(r[1], v.y);
        r[2] = min(r[2], v.z);
        r[3] = min(r[3], v.w);
      }
    }
}

__device__ __forceinline__ void fill_inf(u32 (&c)[8][8]) {
#pragma unroll
  for (int i = 0; i < 8; i++)
#pragma unroll
    for (int j = 0; j < 8; j++) c[i][j] = INF;
}

// The composition runs over a list of group pairs (S1, S2), a chunk of it per
// launch: blockIdx.y = pair plist[pbase + blockIdx.y], whose XT takes slot
// blockIdx.y of the XT buffer (one slot per pair of the chunk).
//
// Workgroups are dealt round-robin to the eight XCDs in order of their linear
// id, so with gridDim.x a multiple of 8 an XCD would get the same tile column
// of every pair; the tiles past a group's last vertex (the padded last
// column, empty for most groups) would then leave one XCD idle.  The tile of
// a workgroup is therefore rotated by its pair.
__device__ __forceinline__ int comp_tile() {
  return (int)((blockIdx.x + blockIdx.y) % gridDim.x);
}

// Positions.  The two-level builds lay each group's vertices out in R, XT
// and the composition's tiles by position: its B2 vertices first (b2list
// order), padding up to a multiple of 4, then its other vertices ascending
// (pos[group * Vrp + p] = local index, -1 for padding).  For y in B2(S2),
// D(S1,S2)[x][y] = XT[y][x]: the first product already holds it (the
// minimum of the second one is reached at b = y, d_S2(y, y) = 0, and no other
// b goes lower, d_S2 being closed), so the first product stores those
// entries and the second one runs only over S2's other vertices.  pos NULL:
// positions are local indices and every column takes the second product.
__device__ __forceinline__ int32_t pos_first(int32_t m2, bool skip) { return skip ? (m2 + 3) & ~3 : 0; }
__device__ __forceinline__ int32_t pos_width(int32_t V, int32_t m2, bool skip) {
  return skip ? ((m2 + 3) & ~3) + V - m2 : V;
}
// local index at position p of a group (base = group * Vrp), -1 for none
__device__ __forceinline__ int32_t pos_local(const int32_t* __restrict__ pos, int64_t base, int32_t p,
                                             int32_t W, int32_t V) {
  if (p >= W) return -1;
  return pos ? pos[base + p] : (p < V ? p : -1);
}

// The certificate's per-wave reduction: largest finite value, and whether
// an INF joins two vertices connected in G.
__device__ __forceinline__ void cert_reduce(u32 best, u32 wrong, u32* cert_bad, u32* cert_mbg) {
  for (int o = 32; o > 0; o >>= 1) {
    best = max(best, (u32)__shfl_xor((int)best, o));
    wrong |= (u32)__shfl_xor((int)wrong, o);
  }
  if ((threadIdx.x & 63) == 0) {
    if (best) atomicMax(cert_mbg, best);
    if (wrong) atomicOr(cert_bad, 1u);
  }
}

// Stores tile c into its block of the query layout, whose element (x, y)
// sits at rowoff(x) |Y| + nb(x) rowoff(y) + loc(x) nb(y) + loc(y) (below
// |X| |Y| < 2^30: 32-bit offsets from the block's base).  Row i of the
// thread is vertex lr[i] of the group whose first BG id is gr (-1: none),
// column j vertex lc[j] of the group at gc.  ROWS_X: c's rows are the
// block's rows x, else its columns y.  CERT: the certificate is folded in.
template <bool CERT, bool ROWS_X>
__device__ __forceinline__ void store_block(const u32 (&c)[8][8], u32* base, int32_t gr, int32_t gc,
                                            const int32_t (&lr)[8], const int32_t (&lc)[8], u32 nY,
                                            const int32_t* __restrict__ bgrow,
                                            const int32_t* __restrict__ bgnb,
                                            const int32_t* __restrict__ bglocal,
                                            const int32_t* __restrict__ bglabel, u32* cert_bad,
                                            u32* cert_mbg) {
  u32 best = 0, wrong = 0;
  // one half of the columns at a time (fewer live registers beside the tile)
#pragma unroll
  for (int h2 = 0; h2 < 2; h2++) {
    // column terms: the block's y terms (rowoff, nb, loc), or with ROWS_X
    // false its x terms (rowoff x |Y|, nb, loc); nb = 0 marks no column
    u32 t0[4], t1[4], t2[4];
    int32_t collab[4];
#pragma unroll
    for (int jj = 0; jj < 4; jj++) {
      const int32_t l = lc[h2 * 4 + jj];
      const int32_t qg = gc + (l >= 0 ? l : 0);
      t0[jj] = ROWS_X ? (u32)bgrow[qg] : (u32)bgrow[qg] * nY;
      t1[jj] = l >= 0 ? (u32)bgnb[qg] : 0u;
      t2[jj] = (u32)bglocal[qg];
      if (CERT) collab[jj] = bglabel[qg];
    }
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (lr[i] < 0) continue;
      const int32_t rg = gr + lr[i];
      const u32 u0 = ROWS_X ? (u32)bgrow[rg] * nY : (u32)bgrow[rg];
      const u32 u1 = (u32)bgnb[rg], u2 = (u32)bglocal[rg];
      const int32_t labr = CERT ? bglabel[rg] : 0;
#pragma unroll
      for (int jj = 0; jj < 4; jj++) {
        if (t1[jj] == 0) continue;
        const u32 v = c[i][h2 * 4 + jj];
        // rowoff(x) |Y| + nb(x) rowoff(y) + loc(x) nb(y) + loc(y)
        const u32 off = ROWS_X ? u0 + __umul24(u1, t0[jj]) + __umul24(u2, t1[jj]) + t2[jj]
                               : t0[jj] + __umul24(t1[jj], u0) + __umul24(t2[jj], u1) + u2;
        base[off] = v;
        if (CERT) {
          if (v < INF) best = max(best, v);
          else wrong |= (u32)(collab[jj] == labr);
        }
      }
    }
  }
  if (CERT) cert_reduce(best, wrong, cert_bad, cert_mbg);
}

// c[i][j] = min(c[i][j], M[lr[i]][lc[j]]) for the valid pairs (M: a group's
// closure, leading dimension ld).
__device__ __forceinline__ void tile_min_gather(u32 (&c)[8][8], const u32* __restrict__ M, int64_t ld,
                                                const int32_t (&lr)[8], const int32_t (&lc)[8]) {
#pragma unroll
  for (int i = 0; i < 8; i++) {
    if (lr[i] < 0) continue;
    const u32* row = M + (int64_t)lr[i] * ld;
#pragma unroll
    for (int j = 0; j < 8; j++)
      if (lc[j] >= 0) c[i][j] = min(c[i][j], row[lc[j]]);
  }
}

// The composition's optional stores (the builds'; the test hooks pass
// none): positions, and the query layout with the certificate or (level 3)
// the dense BG2 matrix.
struct CompStore {
  const int32_t* pos;        // ngroups x Vrp, NULL: identity
  int32_t Vgp, ngroups;      // Mg and b2list leading dimension; groups
  const int32_t *b2list, *gbg0, *bgrow, *bgnb, *bglocal, *bglabel;
  const u32* Mg;
  const int64_t* pairbase;
  u32* H;
  u32 *cert_bad, *cert_mbg;
  // dense store (level 3): element (x, y) of the pair block (S1, S2) at
  // dense[(dbase[S1] + x) * ldo + dbase[S2] + y]; NULL: the query layout
  u32* dense = nullptr;
  int64_t ldo = 0;
  const int32_t* dbase = nullptr;
};

// Stores tile c into a dense matrix: row i of the thread is vertex lr[i]
// (-1: none), column j vertex lc[j], of the groups whose first rows are gx
// (the block's rows) and gy; ROWS_X: c's rows are the block's rows, else its
// columns.
template <bool ROWS_X>
__device__ __forceinline__ void store_dense(const u32 (&c)[8][8], u32* out, int64_t ldo, int64_t gx,
                                            int64_t gy, const int32_t (&lr)[8], const int32_t (&lc)[8]) {
#pragma unroll
  for (int i = 0; i < 8; i++) {
    if (lr[i] < 0) continue;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      if (lc[j] < 0) continue;
      const int64_t off = ROWS_X ? (gx + lr[i]) * ldo + gy + lc[j] : (gx + lc[j]) * ldo + gy + lr[i];
      out[off] = c[i][j];
    }
  }
}

// The first product's entries at S1's B2 positions (positions only):
// XT[b][a] = D2[a][b], the product's minimum taken at a itself
// (d_S1(a, a) = 0; D2 is closed), stored as XT and into the query layout
// (CERT: with the certificate).  One tile: B2 rows ti*128.. of S2 x
// positions tj*128.. of S1; Ab = D2[B2(s1)][B2(s2)] as the product reads it
// (row a, column b, leading dimension lda); sAB holds 8,192 words.
template <bool CERT>
__device__ __forceinline__ void xt_copy_tile(int32_t s1, int32_t s2, bool sw, int ti, int tj,
                                             int32_t ka, int32_t mb, int32_t P1, const u32* Ab,
                                             int64_t lda, u32* xt, int32_t Vrp,
                                             const int32_t* __restrict__ gV, const CompStore& cs,
                                             u32* sAB) {
  const int tx = tid_x(), ty = tid_y();
  u32 c[8][8];
  // c holds rows a (positions tj*128 ..) and columns b, and is stored
  // transposed.  The D2 rows are read whole (a wave reads 256 contiguous
  // bytes), 64 rows at a time through LDS.
  const int32_t bl = (int32_t)threadIdx.x & 127, b = ti * 128 + bl;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    for (int q = 0; q < 32; q++) {
      const int32_t r = 2 * q + ((int32_t)threadIdx.x >> 7), pa = tj * 128 + h * 64 + r;
      sAB[r * 128 + bl] = (pa < ka && b < mb) ? Ab[(int64_t)pa * lda + b] : INF;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int h2 = 0; h2 < 2; h2++) {
        const uint4 v = *reinterpret_cast<const uint4*>(sAB + (ty * 4 + a) * 128 + h2 * 64 + tx * 4);
        c[h * 4 + a][h2 * 4] = v.x;
        c[h * 4 + a][h2 * 4 + 1] = v.y;
        c[h * 4 + a][h2 * 4 + 2] = v.z;
        c[h * 4 + a][h2 * 4 + 3] = v.w;
      }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 8; j++) {
    u32* row = xt + (int64_t)((j >> 2) * 64 + tx * 4 + (j & 3)) * Vrp + tj * 128;
#pragma unroll
    for (int h = 0; h < 2; h++)
      if (tj * 128 + h * 64 + ty * 4 < P1)  // the product's tiles own the rest
        *reinterpret_cast<uint4*>(row + h * 64 + ty * 4) =
            make_uint4(c[h * 4][j], c[h * 4 + 1][j], c[h * 4 + 2][j], c[h * 4 + 3][j]);
  }
  int32_t lr[8], lc[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const int32_t pa = tj * 128 + (i >> 2) * 64 + ty * 4 + (i & 3);
    lr[i] = pa < ka ? cs.pos[(int64_t)s1 * Vrp + pa] : -1;
  }
#pragma unroll
  for (int j = 0; j < 8; j++) {
    const int32_t b = ti * 128 + (j >> 2) * 64 + tx * 4 + (j & 3);
    lc[j] = b < mb ? cs.b2list[(int64_t)s2 * cs.Vgp + b] : -1;
  }
  // D(s1, s2)[a][b] = D2[a][b] (no closure term: d_S1 >= D2 on B2 pairs)
  if (cs.dense) {
    store_dense<true>(c, cs.dense, cs.ldo, cs.dbase[s1], cs.dbase[s2], lr, lc);
    return;
  }
  u32* base = cs.H + (sw ? cs.pairbase[(int64_t)s2 * cs.ngroups + s1]
                         : cs.pairbase[(int64_t)s1 * cs.ngroups + s2]);
  const int32_t gr = cs.gbg0[s1], gc = cs.gbg0[s2];
  if (sw)  // the stored block is (s2, s1): rows (group s1) are its columns
    store_block<CERT, false>(c, base, gr, gc, lr, lc, (u32)gV[s1], cs.bgrow, cs.bgnb, cs.bglocal,
                             cs.bglabel, cs.cert_bad, cs.cert_mbg);
  else
    store_block<CERT, true>(c, base, gr, gc, lr, lc, (u32)gV[s2], cs.bgrow, cs.bgnb, cs.bglocal,
                            cs.bglabel, cs.cert_bad, cs.cert_mbg);
}

// XT (m2pmax x Vrp, rows b in B2(S2), columns: positions of S1) =
//   min over a in B2(S1) of D2[a][b] + R_S1[a][x].
// D2 rows are level-2 ids of the sources (all of BG2, or the share's rows),
// leading dimension ldd.  pstride = 0: D2 is dense (column = level-2 id);
// pstride > 0: D2 is cut into one column panel per group S2, pstride
// elements apart, whose column j is B2(S2)'s j-th vertex: the (S1, S2) block
// a product reads is then one contiguous run instead of rows ldd apart.
// Rows b in [m2[S2], round16(m2[S2])) are stored as INF.  The composition
// reads rows below round16(m2[S2]) and column tiles below S1's width only,
// so tiles past those are neither computed nor written.
//
// A pair flagged PAIR_SWAP reads D2[B2(s1)][B2(s2)] from the transposed
// table D2t (rows: level-2 ids, leading dimension ldt; with a column mask,
// as D2t's columns past B2(s2) belong to other groups).  MODE 1 (2: with the
// certificate) also stores the tile's entries into the query layout, as
// D(s1, s2)[x][y] for y in B2(s2) (D(s2, s1)[y][x] for a swapped pair).
template <int MODE>
__global__ __launch_bounds__(256) SPQ_MP_ATTR void k_mp_xt(const int2* __restrict__ plist, int32_t pbase,
                                               int32_t Vrp, int32_t m2pmax,
                                               const int32_t* __restrict__ m2,
                                               const int32_t* __restrict__ gV,
                                               const int32_t* __restrict__ b2off,
                                               const u32* __restrict__ BG2, int64_t ldd,
                                               int64_t pstride, const u32* __restrict__ D2t,
                                               int64_t ldt,
                                               const u32* __restrict__ R, u32* __restrict__ XT,
                                               CompStore cs) {
  __shared__ __attribute__((aligned(16))) u32 sAB[4 * 16 * 128];
  u32* sA = sAB;
  u32* sB = sAB + 2 * 16 * 128;
  const int2 pr = plist[pbase + (int32_t)blockIdx.y];
  const bool sw = (pr.y & PAIR_SWAP) != 0;
  const int32_t s1 = pr.x, s2 = pr.y & ~PAIR_SWAP;
  const int64_t slot = blockIdx.y;
  const bool skip = cs.pos != nullptr;
  const int ntx = Vrp / 128, ntm = m2pmax / 128;
  // with positions the grid holds twice ntm x ntx tiles: the product's,
  // then as many for S1's B2 positions (copied, see xt_copy_tile), numbered
  // alike, which keeps the product's tile order (the copies as extra
  // columns of each row measured much slower)
  int tile = comp_tile();
  const bool copy = tile >= ntm * ntx;
  if (copy) tile -= ntm * ntx;
  const int ti = tile / ntx, tj = tile % ntx;
  const int32_t ka = m2[s1], mb = m2[s2];
  if (ti * 128 >= mb) return;
  // with positions the product's tiles start past S1's B2 positions
  const int32_t P1 = pos_first(ka, skip), W1 = pos_width(gV[s1], ka, skip);
  // D2[B2(s1)][B2(s2)] as the product reads it (row a, column b)
  const u32* Ab = sw ? D2t + (int64_t)b2off[s1] * ldt + b2off[s2]
                     : BG2 + (int64_t)s2 * pstride + (int64_t)b2off[s1] * ldd + (pstride ? 0 : b2off[s2]);
  const int64_t lda = sw ? ldt : ldd;
  u32* xt = XT + (slot * m2pmax + ti * 128) * Vrp;
  if (MODE > 0 && copy) {
    if (tj * 128 < P1)
      xt_copy_tile<MODE == 2>(s1, s2, sw, ti, tj, ka, mb, P1, Ab, lda, xt, Vrp, gV, cs, sAB);
    return;
  }
  const int tx = tid_x(), ty = tid_y();
  u32 c[8][8];
  const int32_t p0 = P1 + tj * 128;  // first position of the tile
  if (p0 >= W1) return;
  fill_inf(c);
  {
    const u32* B = R + (int64_t)s1 * m2pmax * Vrp + p0;
    // a panel holds INF past its group's B2 vertices: no column mask there
    mp_stream128<true>(c, Ab + ti * 128, lda, B, Vrp, (ka + 15) / 16 * 16, ka,
                       (pstride && !sw) ? 128 : mb - ti * 128, sA, sB, mb - ti * 128, W1 - p0);
  }
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int a = 0; a < 4; a++) {
      const int row = h * 64 + ty * 4 + a;
      const bool live = ti * 128 + row < mb;
#pragma unroll
      for (int h2 = 0; h2 < 2; h2++) {
        const int i = h * 4 + a, j = h2 * 4;
        const int32_t p = p0 + h2 * 64 + tx * 4;  // a multiple of 4: the 4 lie in one row
        if (p >= Vrp) continue;
        uint4 v = live ? make_uint4(c[i][j], c[i][j + 1], c[i][j + 2], c[i][j + 3])
                       : make_uint4(INF, INF, INF, INF);
        *reinterpret_cast<uint4*>(xt + (int64_t)row * Vrp + p) = v;
      }
    }
  if (MODE == 0) return;
  // rows: B2 vertices of s2; columns: positions of s1
  int32_t lr[8], lc[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const int32_t b = ti * 128 + (i >> 2) * 64 + ty * 4 + (i & 3);
    lr[i] = b < mb ? cs.b2list[(int64_t)s2 * cs.Vgp + b] : -1;
  }
#pragma unroll
  for (int j = 0; j < 8; j++)
    lc[j] = pos_local(cs.pos, (int64_t)s1 * Vrp, p0 + (j >> 2) * 64 + tx * 4 + (j & 3), W1, gV[s1]);
  // d_S1 between the two when S1 = S2: d_S1(b, x), the closure being symmetric
  if (s1 == s2) tile_min_gather(c, cs.Mg + (int64_t)s1 * cs.Vgp * cs.Vgp, cs.Vgp, lr, lc);
  if (cs.dense) {  // rows: the block's columns y
    store_dense<false>(c, cs.dense, cs.ldo, cs.dbase[s1], cs.dbase[s2], lr, lc);
    return;
  }
  u32* base = cs.H + (sw ? cs.pairbase[(int64_t)s2 * cs.ngroups + s1]
                         : cs.pairbase[(int64_t)s1 * cs.ngroups + s2]);
  const int32_t gr = cs.gbg0[s2], gc = cs.gbg0[s1];
  if (sw)  // rows (group s2) are the block's rows
    store_block<MODE == 2, true>(c, base, gr, gc, lr, lc, (u32)gV[s1], cs.bgrow, cs.bgnb, cs.bglocal,
                                 cs.bglabel, cs.cert_bad, cs.cert_mbg);
  else
    store_block<MODE == 2, false>(c, base, gr, gc, lr, lc, (u32)gV[s2], cs.bgrow, cs.bgnb, cs.bglocal,
                                  cs.bglabel, cs.cert_bad, cs.cert_mbg);
}

// D(S1,S2) tile for the pair of blockIdx.y, rows at positions of S1, columns
// at positions of S2 past its B2 vertices (all of S2 without positions):
//   min over b in B2(S2) of XT[b][x] + R_S2[b][y], and d_S1 when S1 = S2;
// stored in the component-pair layout described at the top of the file.
// CERT: the exactness certificate is fused into the store.
template <bool CERT>
__global__ __launch_bounds__(256) SPQ_MP_ATTR void k_mp_y(const int2* __restrict__ plist, int32_t pbase,
                                              int32_t Vrp, int32_t m2pmax,
                                              const int32_t* __restrict__ m2,
                                              const int32_t* __restrict__ gV,
                                              const u32* __restrict__ XT, const u32* __restrict__ R,
                                              CompStore cs) {
  __shared__ __attribute__((aligned(16))) u32 sA[2 * 16 * 128];
  __shared__ __attribute__((aligned(16))) u32 sB[2 * 16 * 128];
  const int2 pr = plist[pbase + (int32_t)blockIdx.y];
  const bool sw = (pr.y & PAIR_SWAP) != 0;
  const int32_t s1 = pr.x, s2 = pr.y & ~PAIR_SWAP;
  const int64_t slot = blockIdx.y;
  const int ntx = Vrp / 128;
  const int tile = comp_tile();
  const int ti = tile / ntx, tj = tile % ntx;
  const bool skip = cs.pos != nullptr;
  const int32_t V1 = gV[s1], V2 = gV[s2], kb = m2[s2];
  const int32_t W1 = pos_width(V1, m2[s1], skip), W2 = pos_width(V2, kb, skip);
  const int32_t c0 = pos_first(kb, skip) + tj * 128;  // first column position of the tile
  if (ti * 128 >= W1 || c0 >= W2) return;
  u32 c[8][8];
  fill_inf(c);
  const u32* At = XT + slot * m2pmax * Vrp + ti * 128;
  const u32* B = R + (int64_t)s2 * m2pmax * Vrp + c0;
  mp_stream128<false>(c, At, Vrp, B, Vrp, (kb + 15) / 16 * 16, kb, 0, sA, sB, W1 - ti * 128,
                      W2 - c0);
  const int tx = tid_x(), ty = tid_y();
  int32_t lr[8], lc[8];
#pragma unroll
  for (int i = 0; i < 8; i++)
    lr[i] = pos_local(cs.pos, (int64_t)s1 * Vrp, ti * 128 + (i >> 2) * 64 + ty * 4 + (i & 3), W1, V1);
#pragma unroll
  for (int j = 0; j < 8; j++)
    lc[j] = pos_local(cs.pos, (int64_t)s2 * Vrp, c0 + (j >> 2) * 64 + tx * 4 + (j & 3), W2, V2);
  // the group's own closure when S1 = S2, folded in after the product:
  // taken in first, it kept a second copy of the tile live through the K loop
  if (s1 == s2) tile_min_gather(c, cs.Mg + (int64_t)s1 * cs.Vgp * cs.Vgp, cs.Vgp, lr, lc);
  u32* base = cs.H + (sw ? cs.pairbase[(int64_t)s2 * cs.ngroups + s1]
                         : cs.pairbase[(int64_t)s1 * cs.ngroups + s2]);
  const int32_t gr = cs.gbg0[s1], gc = cs.gbg0[s2];
  if (sw)  // the stored block is (s2, s1): rows of s1 are its columns
    store_block<CERT, false>(c, base, gr, gc, lr, lc, (u32)V1, cs.bgrow, cs.bgnb, cs.bglocal,
                             cs.bglabel, cs.cert_bad, cs.cert_mbg);
  else
    store_block<CERT, true>(c, base, gr, gc, lr, lc, (u32)V2, cs.bgrow, cs.bgnb, cs.bglocal,
                            cs.bglabel, cs.cert_bad, cs.cert_mbg);
}

// ------------------------------------------------------------- level 3
// The construction once more, on BG2, when BG2 itself is too large for one
// flat Floyd-Warshall: super-groups T of consecutive groups; M3[T] = BG2
// induced on T's vertices, closed (d_T); B3(T) = vertices of T with a G edge
// to another super-group (the only BG2 edges that leave T); BG3 on the B3
// vertices, closed by flat Floyd-Warshall (= d_BG2 on B3, Lemma 1 for the
// super-group partition); then, by Lemma 3 at this level,
//   d_BG2(x,y) = min over a in B3(T1), b in B3(T2) of
//                d_T1(x,a) + d_BG3(a,b) + d_T2(b,y)   (and d_T1(x,y) if T1 = T2),
// evaluated with the same two products and written straight into the dense
// BG2 matrix for T1 <= T2: the block upper triangle the level-2 composition
// reads (rows of a group S1, columns of a group S2 >= S1).

// M3[T] (V3gp x V3gp): T's block of the unclosed BG2 matrix; 0 on the
// padding's diagonal, INF elsewhere on the padding.
__global__ void k_l3_gather(int64_t V2p, const u32* __restrict__ BG2, const int32_t* __restrict__ tbase,
                            const int32_t* __restrict__ tsize, int32_t V3gp, u32* __restrict__ M3) {
  const int t = blockIdx.y;
  const int64_t p = blockIdx.x;
  const int32_t nt = tsize[t];
  u32* out = M3 + ((int64_t)t * V3gp + p) * V3gp;
  const u32* src = BG2 + ((int64_t)tbase[t] + p) * V2p + tbase[t];
  for (int64_t q0 = (int64_t)threadIdx.x * 4; q0 < V3gp; q0 += (int64_t)blockDim.x * 4) {
    u32 v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int64_t q = q0 + u;
      v[u] = (p < nt && q < nt) ? src[q] : (q == p ? 0u : INF);
    }
    *reinterpret_cast<uint4*>(out + q0) = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

// G edges between super-groups (both ends are level-2 vertices).  BG3 ==
// NULL: flags both ends as level-3 boundary vertices; otherwise enters the
// edge into BG3 (ids b3off[T] + rank inside T).
__global__ void k_l3_edges(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                           const int32_t* __restrict__ w, const int32_t* __restrict__ comp,
                           const int32_t* __restrict__ local, const int32_t* __restrict__ bgoff,
                           const int32_t* __restrict__ grp, int32_t gpt, const int32_t* __restrict__ b2off,
                           const int32_t* __restrict__ b2rank, uint8_t* __restrict__ flag3,
                           const int32_t* __restrict__ b3off, const int32_t* __restrict__ b3rank,
                           int64_t V3p, u32* __restrict__ BG3) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = eu[e], v = ev[e];
    const int32_t cu = comp[u], cv = comp[v];
    if (cu == cv) continue;
    const int32_t su = grp[cu], sv = grp[cv];
    const int32_t tu = su / gpt, tv = sv / gpt;
    if (tu == tv) continue;
    const int32_t xu = b2off[su] + b2rank[bgoff[cu] + local[u]];
    const int32_t xv = b2off[sv] + b2rank[bgoff[cv] + local[v]];
    if (!BG3) {
      flag3[xu] = 1;
      flag3[xv] = 1;
      continue;
    }
    const int64_t a = b3off[tu] + b3rank[xu], b = b3off[tv] + b3rank[xv];
    atomicMin(BG3 + a * V3p + b, (u32)w[e]);
    atomicMin(BG3 + b * V3p + a, (u32)w[e]);
  }
}

// D_BG2 tile for the super-group pair of blockIdx.y (T1 <= T2), rows at
// positions of T1, columns at positions of T2 past its B3 vertices (all of
// T2 without positions, pos NULL), into the dense matrix out (leading
// dimension ldo, rows and columns from the super-groups' first BG2 ids
// gbase).  XT and R have rows Vrp words long; Mg (the closures, leading
// dimension Vgp) is folded in when T1 = T2.
__global__ __launch_bounds__(256) SPQ_MP_ATTR void k_mp_y_dense(const int2* __restrict__ plist, int32_t pbase,
                                                    int32_t Vgp, int32_t Vrp,
                                                    int32_t m2pmax, const int32_t* __restrict__ m2,
                                                    const int32_t* __restrict__ gV,
                                                    const int32_t* __restrict__ gbase,
                                                    const int32_t* __restrict__ pos,
                                                    const u32* __restrict__ XT, const u32* __restrict__ R,
                                                    const u32* __restrict__ Mg, u32* __restrict__ out,
                                                    int64_t ldo) {
  __shared__ __attribute__((aligned(16))) u32 sA[2 * 16 * 128];
  __shared__ __attribute__((aligned(16))) u32 sB[2 * 16 * 128];
  const int2 pr = plist[pbase + (int32_t)blockIdx.y];
  const int32_t s1 = pr.x, s2 = pr.y;
  const int64_t slot = blockIdx.y;
  const int ntx = Vrp / 128;
  const int tile = comp_tile();
  const int ti = tile / ntx, tj = tile % ntx;
  const bool skip = pos != nullptr;
  const int32_t V1 = gV[s1], V2 = gV[s2], kb = m2[s2];
  const int32_t W1 = pos_width(V1, m2[s1], skip), W2 = pos_width(V2, kb, skip);
  const int32_t c0 = pos_first(kb, skip) + tj * 128;  // first column position of the tile
  if (ti * 128 >= W1 || c0 >= W2) return;
  u32 c[8][8];
  fill_inf(c);
  const u32* At = XT + slot * m2pmax * Vrp + ti * 128;
  const u32* B = R + (int64_t)s2 * m2pmax * Vrp + c0;
  mp_stream128<false>(c, At, Vrp, B, Vrp, (kb + 15) / 16 * 16, kb, 0, sA, sB, W1 - ti * 128,
                      W2 - c0);
  const int tx = tid_x(), ty = tid_y();
  int32_t lr[8], lc[8];
#pragma unroll
  for (int i = 0; i < 8; i++)
    lr[i] = pos_local(pos, (int64_t)s1 * Vrp, ti * 128 + (i >> 2) * 64 + ty * 4 + (i & 3), W1, V1);
#pragma unroll
  for (int j = 0; j < 8; j++)
    lc[j] = pos_local(pos, (int64_t)s2 * Vrp, c0 + (j >> 2) * 64 + tx * 4 + (j & 3), W2, V2);
  // the super-group's own closure when T1 = T2, folded in after the product
  if (s1 == s2) tile_min_gather(c, Mg + (int64_t)s1 * Vgp * Vgp, Vgp, lr, lc);
  store_dense<true>(c, out, ldo, gbase[s1], gbase[s2], lr, lc);
}

// One BG row (BG id x) gathered from the two-level store, for inspection.
__global__ void k_hier_row(int32_t x, int32_t swap, int32_t V, int32_t ngroups,
                           const int32_t* __restrict__ bggrp,
                           const int32_t* __restrict__ bgrow, const int32_t* __restrict__ bgnb,
                           const int32_t* __restrict__ bglocal, const int32_t* __restrict__ gV,
                           const int64_t* __restrict__ pairbase, const u32* __restrict__ H,
                           u32* __restrict__ out) {
  const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= V) return;
  int32_t a = x, b = (int32_t)y;
  if (swap && bggrp[a] > bggrp[b]) {
    a = (int32_t)y;
    b = x;
  }
  const int32_t sa = bggrp[a], sb = bggrp[b];
  const int64_t off = pairbase[(int64_t)sa * ngroups + sb] + (int64_t)bgrow[a] * gV[sb] +
                      (int64_t)bgnb[a] * bgrow[b] + (int64_t)bglocal[a] * bgnb[b] + bglocal[b];
  out[y] = H[off];
}


// ------------------------------------------------------------ share mode --
// Distances from the level-2 boundary vertices of the share groups (the
// first share_groups groups; their level-2 ids are 0 .. S2-1) to all level-2
// vertices, by Bellman-Ford over blocks of consecutive groups on BG2, without
// building BG2.  A block T is a run of consecutive groups (one group: the
// Bellman-Ford over groups); A_T = BG2 induced on T's level-2 vertices (d_S
// between the B2
// vertices of one group S, the G edges between groups of T), closed.  DT[b][i]
// (row b = any level-2 id, column i = share source) alternates
//   intra-block:  DT[T] = min(DT[T], A_T (x) DT[T])   (A_T closed: one product
//                 covers any walk that stays inside T)
//   cross edges:  DT[b] = min(DT[b], DT[a] + w(a,b))  for each G edge between blocks
// until nothing changes.  Every walk of BG2 is a sequence of pieces inside one
// block joined by G edges between blocks, so the fixed point is d_BG2 from
// every share source (Lemma 1 for the block partition of BG2).  Larger blocks
// mean fewer rounds (a round crosses one block) and fewer cross edges, at the
// price of larger products.

// A_T before its closure (bpmax x bpmax per block, local level-2 indices):
// d_S between the B2 vertices of one group, 0 on the diagonal, INF elsewhere
// and on the padding.  Block t holds groups [bfirst[t], bfirst[t+1]); a block
// of one group: A_T = d_S on B2(S), already closed.
__global__ void k_blk_init(int32_t Vgp, int32_t bpmax, const int32_t* __restrict__ bfirst,
                           const int32_t* __restrict__ b2off, const int32_t* __restrict__ b2list,
                           const u32* __restrict__ Mg, u32* __restrict__ A) {
  const int t = blockIdx.y;
  const int32_t p = blockIdx.x;
  const int32_t g0 = bfirst[t], g1 = bfirst[t + 1];
  const int32_t base = b2off[g0], size = b2off[g1] - base;
  u32* out = A + ((int64_t)t * bpmax + p) * bpmax;
  int32_t lo = 0, hi = 0;
  const u32* prow = nullptr;
  const int32_t* list = nullptr;
  if (p < size) {
    int32_t a = g0;  // the row's group (a block holds few groups)
    while (a + 1 < g1 && b2off[a + 1] - base <= p) a++;
    lo = b2off[a] - base;
    hi = b2off[a + 1] - base;
    list = b2list + (int64_t)a * Vgp;
    prow = Mg + ((int64_t)a * Vgp + list[p - lo]) * Vgp;
  }
  for (int32_t q = threadIdx.x; q < bpmax; q += blockDim.x)
    out[q] = (q == p) ? 0u : (q >= lo && q < hi) ? prow[list[q - lo]] : INF;
}

// G edges between groups of the same block, into A_T (both directions).
__global__ void k_blk_edges(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            const int32_t* __restrict__ w, const int32_t* __restrict__ comp,
                            const int32_t* __restrict__ local, const int32_t* __restrict__ bgoff,
                            const int32_t* __restrict__ grp, const int32_t* __restrict__ gblk,
                            const int32_t* __restrict__ bfirst,
                            const int32_t* __restrict__ b2off, const int32_t* __restrict__ b2rank,
                            int32_t bpmax, u32* __restrict__ A) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = eu[e], v = ev[e];
    const int32_t cu = comp[u], cv = comp[v];
    if (cu == cv) continue;
    const int32_t su = grp[cu], sv = grp[cv];
    if (su == sv || gblk[su] != gblk[sv]) continue;
    const int32_t t = gblk[su], base = b2off[bfirst[t]];
    const int64_t a = b2off[su] + b2rank[bgoff[cu] + local[u]] - base;
    const int64_t b = b2off[sv] + b2rank[bgoff[cv] + local[v]] - base;
    u32* At = A + (int64_t)t * bpmax * bpmax;
    atomicMin(At + a * bpmax + b, (u32)w[e]);
    atomicMin(At + b * bpmax + a, (u32)w[e]);
  }
}

// DT init: row b (level-2 id), column i (share source): the distance inside
// b's block when i lies in it (row b of the closed A_T), 0 for b = i, INF
// otherwise.  boff: first level-2 id of each block (nblk + 1 entries).
__global__ void k_dt_init(int32_t V2, int32_t S2, int64_t S2p, int32_t nblk,
                          const int32_t* __restrict__ boff, int32_t bpmax, const u32* __restrict__ A,
                          u32* __restrict__ DT) {
  const int64_t b = blockIdx.x;
  u32* out = DT + b * S2p;
  int64_t lo = 0, hi = 0;
  const u32* arow = nullptr;
  if (b < V2) {
    int32_t a = 0, z = nblk - 1;
    while (a < z) {
      const int32_t mid = (a + z + 1) >> 1;
      if (boff[mid] <= b) a = mid; else z = mid - 1;
    }
    lo = boff[a];
    hi = min((int64_t)boff[a + 1], (int64_t)S2);
    arow = A + ((int64_t)a * bpmax + (b - lo)) * bpmax;
  }
  for (int64_t i = threadIdx.x; i < S2p; i += blockDim.x)
    out[i] = (i == b) ? 0u : (i >= lo && i < hi) ? arow[i - lo] : INF;
}

// Dirty flags of the Bellman-Ford rounds: per block (a group or a run of
// groups), one word per column tile of 128 share sources, then one word "any
// tile" (stride ntc + 1).  Beside them, per (block, column tile), the B3 rows
// (indices in the block's b3list) that the cross edges lowered since the
// block's last intra step: a count and a list (count BF_ALL_ROWS: every row).
//
// Intra-block step, in place: the block's rows x column tile of DT = min(DT,
// A (x) DT) for the (block, tile) pairs whose values changed in the previous
// round.  One product with the closed A leaves the rows closed.  The rows were
// closed before the cross edges lowered some of them, and for an unchanged
// row k, A[x][k] + DT[k] >= DT[x] already; so only the lowered rows need to
// be the K of the product.  Tiles of one block read rows that other tiles of
// the block are lowering: every value read is the old or the new one, both
// lengths of real walks and each at most the old value, and A being closed,
// the old values already give the closed result, so the step is exact in any
// interleaving.  The rounds run this step on the B3 rows only (k_bf_intra3
// below, with A restricted to B3 x B3, which is closed as well: a shortest
// path inside the block between two B3 vertices needs no other row of DT).

// Cross edges between blocks, as directed level-2 pairs (a -> b, w), tagged
// (source block << 16) | destination block.
__global__ void k_cross_collect(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                                const int32_t* __restrict__ w, const int32_t* __restrict__ comp,
                                const int32_t* __restrict__ local, const int32_t* __restrict__ bgoff,
                                const int32_t* __restrict__ grp, const int32_t* __restrict__ gblk,
                                const int32_t* __restrict__ b2off,
                                const int32_t* __restrict__ b2rank, int32_t* __restrict__ count,
                                int4* __restrict__ xe) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = eu[e], v = ev[e];
    const int32_t cu = comp[u], cv = comp[v];
    if (cu == cv) continue;
    const int32_t su = grp[cu], sv = grp[cv];
    const int32_t tu = gblk[su], tv = gblk[sv];  // blocks
    if (tu == tv) continue;
    const int32_t a = b2off[su] + b2rank[bgoff[cu] + local[u]];
    const int32_t b = b2off[sv] + b2rank[bgoff[cv] + local[v]];
    const int32_t slot = atomicAdd(count, 2);
    xe[slot] = make_int4(a, b, w[e], (tu << 16) | tv);
    xe[slot + 1] = make_int4(b, a, w[e], (tv << 16) | tu);
  }
}

// DT[b][i] = min(DT[b][i], DT[a][i] + w) for every directed cross edge, on
// the column tiles that are dirty for the source block (values that have not
// changed since they were last propagated need no new pass); a lowered value
// marks its (block, tile) dirty for the next round and, once per round (the
// stamp of (row, tile) holds the round that last listed it), adds its row to
// that (block, tile)'s list as its index among the block's B3 rows (b3rank;
// a cross edge ends in B3 by definition; lstride: list slots per (block,
// tile)).
__global__ void k_bf_cross(int32_t nxe, const int4* __restrict__ xe, int32_t S2, int64_t S2p, u32* DT,
                           const u32* __restrict__ dirty, u32* __restrict__ dirty_next,
                           const int32_t* __restrict__ b3rank, int32_t lstride, u32 round,
                           u32* __restrict__ stamp, int32_t* __restrict__ rcnt_next,
                           int32_t* __restrict__ rlist_next) {
  const int32_t e = blockIdx.x;
  if (e >= nxe) return;
  const int4 t = xe[e];
  const int ntc = (int)(S2p / 128);
  const u32* dsrc = dirty + (int64_t)(t.w >> 16) * (ntc + 1);
  if (!dsrc[ntc]) return;
  const int32_t sv = t.w & 0xffff;
  u32* dnext = dirty_next + (int64_t)sv * (ntc + 1);
  const u32* src = DT + (int64_t)t.x * S2p;
  u32* dst = DT + (int64_t)t.y * S2p;
  // tiles this workgroup has already listed its row for (LDS, when they fit):
  // the global stamp is then touched once per tile, not once per element
  __shared__ u32 listed[BF_LDS_TILES];
  const bool local = ntc <= BF_LDS_TILES;
  if (local) {
    for (int q = threadIdx.x; q < ntc; q += blockDim.x) listed[q] = 0u;
    __syncthreads();
  }
  // four consecutive columns per thread and step (one 16-byte load of each
  // row; rows are S2p words apart, a multiple of 128, and the four lie in
  // one column tile)
  for (int32_t i0 = 4 * (int32_t)threadIdx.x; i0 < S2; i0 += 4 * (int32_t)blockDim.x) {
    const int tile = i0 >> 7;
    if (!dsrc[tile]) continue;
    const uint4 a4 = *reinterpret_cast<const uint4*>(src + i0);
    const uint4 d4 = *reinterpret_cast<const uint4*>(dst + i0);
    const u32 av[4] = {a4.x, a4.y, a4.z, a4.w}, dv[4] = {d4.x, d4.y, d4.z, d4.w};
    bool lowered = false;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const u32 v = min(av[q] + (u32)t.z, INF);
      if (i0 + q < S2 && v < dv[q]) {
        atomicMin(dst + i0 + q, v);
        lowered = true;
      }
    }
    if (!lowered) continue;
    dnext[tile] = 1u;
    dnext[ntc] = 1u;
    if (local && atomicExch(listed + tile, 1u) != 0u) continue;
    if (atomicExch(stamp + (int64_t)t.y * ntc + tile, round) != round) {
      const int64_t st = (int64_t)sv * ntc + tile;
      const int32_t slot = atomicAdd(rcnt_next + st, 1);
      rlist_next[st * lstride + slot] = b3rank[t.y];
    }
  }
}

// ------------------------------------------------------------- block boundary
// Only the B3 rows of a block (level-2 vertices with a G edge to another
// block) are lowered by cross edges and read by them, so the rounds keep
// just those rows settled; a path from a source to any other row v of block
// T either stays in T (DT's initial row, from the closed A_T) or enters T
// last through some b in B3(T), so once the B3 rows are exact
//   DT[v] = min(DT[v], min over b in B3(T) of A_T[v][b] + DT[b])
// gives the rest in one product per block.

// flag3[a] = 1 for every source a of a directed cross edge (both directions
// are listed, so every endpoint); the count is read on the device.
__global__ void k_b3_mark(const int32_t* __restrict__ xcount, const int4* __restrict__ xe,
                          uint8_t* __restrict__ flag3) {
  const int32_t n = *xcount;
  for (int32_t e = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); e < n;
       e += (int32_t)(gridDim.x * blockDim.x))
    flag3[xe[e].x] = 1;
}

__global__ void k_flag_not(int32_t n, const uint8_t* __restrict__ f, uint8_t* __restrict__ g) {
  for (int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); i < n;
       i += (int32_t)(gridDim.x * blockDim.x))
    g[i] = f[i] ? 0 : 1;
}

// Row i of block t's A3: A_T[b3[i]][b3[j]] for i, j < m3[t]; INF elsewhere.
__global__ void k_a3_gather(int32_t bpmax, int32_t b3pmax, const int32_t* __restrict__ m3,
                            const int32_t* __restrict__ b3list, const u32* __restrict__ A,
                            u32* __restrict__ A3) {
  const int t = blockIdx.y;
  const int32_t i = blockIdx.x, mt = m3[t];
  const int32_t* bl = b3list + (int64_t)t * bpmax;
  u32* out = A3 + ((int64_t)t * b3pmax + i) * b3pmax;
  const u32* arow = i < mt ? A + ((int64_t)t * bpmax + bl[i]) * bpmax : nullptr;
  for (int32_t j = threadIdx.x; j < b3pmax; j += blockDim.x) out[j] = (arow && j < mt) ? arow[bl[j]] : INF;
}

// Row k of block t's Aout: A_T[b3[k]][nb3[i]] for k < m3[t], i < n3[t]; INF
// elsewhere (A_T is symmetric: row b3[k] holds column b3[k]).
__global__ void k_aout_gather(int32_t bpmax, int32_t b3pmax, int32_t n3pmax,
                              const int32_t* __restrict__ m3, const int32_t* __restrict__ n3,
                              const int32_t* __restrict__ b3list, const int32_t* __restrict__ nb3list,
                              const u32* __restrict__ A, u32* __restrict__ Aout) {
  const int t = blockIdx.y;
  const int32_t k = blockIdx.x, nt = n3[t];
  const int32_t* bl = b3list + (int64_t)t * bpmax;
  const int32_t* nl = nb3list + (int64_t)t * bpmax;
  u32* out = Aout + ((int64_t)t * b3pmax + k) * n3pmax;
  const u32* arow = k < m3[t] ? A + ((int64_t)t * bpmax + bl[k]) * bpmax : nullptr;
  for (int32_t i = threadIdx.x; i < n3pmax; i += blockDim.x) out[i] = (arow && i < nt) ? arow[nl[i]] : INF;
}

// The 128 x 128 tile whose row r is g + rows[r] * ld, in the register layout
// of tile_load; rows r >= nvalid read as INF and are not stored.
__device__ __forceinline__ void tile_load_rows(u32 (&c)[8][8], const u32* g, int64_t ld,
                                               const int32_t* __restrict__ rows, int nvalid) {
  const int tx = tid_x(), ty = tid_y();
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int a = 0; a < 4; a++) {
      const int r = h * 64 + ty * 4 + a;
      if (r < nvalid) {
        const u32* row = g + (int64_t)rows[r] * ld + tx * 4;
#pragma unroll
        for (int h2 = 0; h2 < 2; h2++) {
          const uint4 v = *reinterpret_cast<const uint4*>(row + h2 * 64);
          u32* d = c[h * 4 + a] + h2 * 4;
          d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; j++) c[h * 4 + a][j] = INF;
      }
    }
}

__device__ __forceinline__ void tile_store_rows(const u32 (&c)[8][8], u32* g, int64_t ld,
                                                const int32_t* __restrict__ rows, int nvalid) {
  const int tx = tid_x(), ty = tid_y();
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int a = 0; a < 4; a++) {
      const int r = h * 64 + ty * 4 + a;
      if (r >= nvalid) continue;
      u32* row = g + (int64_t)rows[r] * ld + tx * 4;
#pragma unroll
      for (int h2 = 0; h2 < 2; h2++) {
        const u32* v = c[h * 4 + a] + h2 * 4;
        *reinterpret_cast<uint4*>(row + h2 * 64) = make_uint4(v[0], v[1], v[2], v[3]);
      }
    }
}

// The intra-block step of a round on the B3 rows only (see the Intra-block
// step above for why the listed rows suffice and why in place is exact): rows
// b3[ti*128 ..] x column tile tj of block s = min(DT, A3 (x) DT) over the
// listed B3 rows (their indices in b3list).
__global__ __launch_bounds__(256) void k_bf_intra3(int32_t bpmax, int32_t b3pmax, int64_t S2p,
                                                   const int32_t* __restrict__ m3,
                                                   const int32_t* __restrict__ boff,
                                                   const int32_t* __restrict__ b3list,
                                                   const u32* __restrict__ A3, u32* DT,
                                                   const u32* __restrict__ dirty,
                                                   const int32_t* __restrict__ rcnt,
                                                   const int32_t* __restrict__ rlist) {
  __shared__ __attribute__((aligned(16))) u32 sA[2 * 16 * 128];
  __shared__ __attribute__((aligned(16))) u32 sB[2 * 16 * 128];
  const int s = blockIdx.y;
  const int32_t ms = m3[s];
  const int ntc = (int)(S2p / 128);
  const int ti = (int)blockIdx.x / ntc, tj = (int)blockIdx.x % ntc;
  if (ti * 128 >= ms || !dirty[(int64_t)s * (ntc + 1) + tj]) return;
  const int64_t st = (int64_t)s * ntc + tj;
  const int32_t cnt = rcnt[st];
  if (cnt == 0) return;
  const int32_t* bl = b3list + (int64_t)s * bpmax;
  u32* D = DT + (int64_t)boff[s] * S2p + tj * 128;  // the block's rows, this column tile
  const int nv = min(128, ms - ti * 128);
  u32 c[8][8];
  tile_load_rows(c, D, S2p, bl + ti * 128, nv);
  const u32* At = A3 + (int64_t)s * b3pmax * b3pmax + ti * 128;  // symmetric: At[k][i] = A3[i][k]
  const bool all = cnt == BF_ALL_ROWS;
  mp_stream128_rows(c, At, b3pmax, D, S2p, all ? nullptr : rlist + st * b3pmax, all ? ms : cnt, sA, sB,
                    bl);
  tile_store_rows(c, D, S2p, bl + ti * 128, nv);
}

// The rows outside B3, once the rounds have settled: rows nb3[ti*128 ..] x
// column tile tj of block s = min(DT, Aout^T (x) DT[B3 rows]).
__global__ __launch_bounds__(256) void k_bf_final(int32_t bpmax, int32_t b3pmax, int32_t n3pmax,
                                                  int64_t S2p, const int32_t* __restrict__ m3,
                                                  const int32_t* __restrict__ n3,
                                                  const int32_t* __restrict__ boff,
                                                  const int32_t* __restrict__ b3list,
                                                  const int32_t* __restrict__ nb3list,
                                                  const u32* __restrict__ Aout, u32* DT) {
  __shared__ __attribute__((aligned(16))) u32 sA[2 * 16 * 128];
  __shared__ __attribute__((aligned(16))) u32 sB[2 * 16 * 128];
  const int s = blockIdx.y;
  const int32_t nn = n3[s], kk = m3[s];
  const int ntc = (int)(S2p / 128);
  const int ti = (int)blockIdx.x / ntc, tj = (int)blockIdx.x % ntc;
  if (ti * 128 >= nn || kk == 0) return;
  const int32_t* nl = nb3list + (int64_t)s * bpmax;
  u32* D = DT + (int64_t)boff[s] * S2p + tj * 128;
  const int nv = min(128, nn - ti * 128);
  u32 c[8][8];
  tile_load_rows(c, D, S2p, nl + ti * 128, nv);
  const u32* At = Aout + (int64_t)s * b3pmax * n3pmax + ti * 128;  // At[k][i] = A_T[b3[k]][nb3[i]]
  mp_stream128_rows(c, At, n3pmax, D, S2p, nullptr, kk, sA, sB, b3list + (int64_t)s * bpmax);
  tile_store_rows(c, D, S2p, nl + ti * 128, nv);
}

// The share's D2 in column panels: panel S (one per group, S2p x m2pmax
// elements) holds D2[i][j] = DT[b2off[S] + j][i] for the share sources i and
// the B2(S) vertices j < m2[S], INF in the columns past m2[S].  32 x 32 tiles
// through LDS; blockIdx.z = the group.
__global__ void k_panel_transpose(const u32* __restrict__ DT, int64_t S2p, int32_t m2pmax,
                                  const int32_t* __restrict__ m2, const int32_t* __restrict__ b2off,
                                  u32* __restrict__ D2) {
  __shared__ u32 t[32][33];
  const int g = blockIdx.z;
  const int32_t ms = m2[g], r0 = b2off[g];
  const int64_t i0 = (int64_t)blockIdx.x * 32;  // share sources (panel rows)
  const int32_t j0 = (int32_t)blockIdx.y * 32;  // B2(S) vertices (panel columns)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8)
    if (j0 + k < ms && i0 + tx < S2p) t[k][tx] = DT[(int64_t)(r0 + j0 + k) * S2p + i0 + tx];
  __syncthreads();
  u32* panel = D2 + (int64_t)g * S2p * m2pmax;
  for (int k = ty; k < 32; k += 8)
    if (i0 + k < S2p) panel[(i0 + k) * m2pmax + j0 + tx] = j0 + tx < ms ? t[tx][k] : INF;
}

// ---------------------------------------------------------------- launch --
static inline unsigned hblocks(int64_t items) {
  int64_t b = (items + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (unsigned)b;
}

hipError_t launch_hier_level1(const HierArgs& a, hipStream_t s) {
  k_hier_vmeta<<<hblocks(a.V), 256, 0, s>>>(a.V, a.bgcomp, a.bgoff, a.nb, a.grp, a.gbg0,
                                                              a.bgrow, a.bgnb, a.bggrp);
  k_grp_init<<<dim3((unsigned)a.Vgp, (unsigned)a.ngroups), 256, 0, s>>>(
      a.Vgp, a.gbg0, a.gV, a.bgcomp, a.bglocal, a.bgoff, a.nb, a.P, a.moff, a.M, a.Mg);
  if (a.m > 0)
    k_grp_edges<<<hblocks(a.m), 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.comp, a.local, a.bgoff, a.grp,
                                             a.gbg0, a.Vgp, a.Mg, a.flag2);
  const int ntg = a.Vgp / 128;
  hipError_t e = (a.side && ntg > 1)
                     ? launch_dense_fw_batch_lookahead(a.Mg, a.Vgp, 128, ntg, a.ngroups,
                                                       (int64_t)a.Vgp * a.Vgp, s, a.side, a.sync,
                                                       nullptr, a.kc, a.pivot)
                     : launch_dense_fw_batch(a.Mg, a.Vgp, 128, ntg, a.ngroups, (int64_t)a.Vgp * a.Vgp,
                                             s, nullptr, a.kc, a.pivot);
  if (e != hipSuccess) return e;
  k_b2_scan<<<(unsigned)a.ngroups, 256, 0, s>>>(a.gbg0, a.gV, a.flag2, a.Vgp, a.b2list, a.b2rank, a.m2);
  return hipGetLastError();
}

// The groups' positions and R_S by position.
static void launch_rpos(const HierArgs& a, hipStream_t s) {
  k_pos_build<<<(unsigned)a.ngroups, 256, 0, s>>>(a.gbg0, a.gV, a.b2rank, a.b2list, a.m2, a.Vgp, a.Vrp,
                                                  a.pos);
  k_rpos_gather<<<dim3((unsigned)a.m2pmax, (unsigned)a.ngroups), 256, 0, s>>>(
      a.Vgp, a.Vrp, a.m2pmax, a.m2, a.b2list, a.pos, a.Mg, a.R);
}

hipError_t launch_hier_level2_prep(const HierArgs& a, hipStream_t s) {
  launch_rpos(a, s);
  if (a.V2p > 0) {
    k_bg2_init<<<(unsigned)a.V2p, 256, 0, s>>>(a.V2, a.V2p, a.ngroups, a.b2off, a.b2list, a.Vgp, a.Mg,
                                               a.BG2);
    if (a.m > 0)
      k_bg2_edges<<<hblocks(a.m), 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.comp, a.local, a.bgoff, a.grp,
                                               a.b2off, a.b2rank, a.V2p, a.BG2);
  }
  return hipGetLastError();
}

hipError_t launch_hier_level2_close(const HierArgs& a, hipStream_t s) {
  if (a.V2p <= 0) return hipSuccess;
  const int nt = (int)(a.V2p / 128);
  if (a.side && nt > 1)
    return launch_dense_fw_lookahead(a.BG2, a.V2p, 128, nt, s, a.side, a.sync, nullptr, a.kc, a.pivot);
  return launch_dense_fw(a.BG2, a.V2p, 128, nt, s, nullptr, a.kc, a.pivot);
}

// Composition over the pair list a.plist (a.npairs pairs), a.chunk pairs per
// launch of each product.  evt (optional) gets a pair of events around every
// k_mp_y launch.  The share's BG2 rows come from its Bellman-Ford (DT^T).
static hipError_t compose_level2(const HierArgs& a, const int32_t* bglabel, u32* cert_bad,
                                 u32* cert_mbg, hipStream_t s) {
  const int32_t Vrp = a.pos ? a.Vrp : a.Vgp;
  const int ntx = Vrp / 128, ntm = a.m2pmax / 128;
  const CompStore cs{a.pos,     a.Vgp,    a.ngroups, a.b2list, a.gbg0,   a.bgrow,  a.bgnb,
                     a.bglocal, bglabel,  a.Mg,      a.pairbase, a.H,    cert_bad, cert_mbg};
  const int64_t ldd = a.d2pstride ? a.d2ld : a.V2p;
  for (int32_t p0 = 0, c = 0; p0 < a.npairs; p0 += a.chunk, c++) {
    const unsigned np = (unsigned)min(a.chunk, a.npairs - p0);
    // with positions the first product's grid holds the copied tiles too
    const dim3 gx((unsigned)(ntm * ntx * (a.pos ? 2 : 1)), np), gy((unsigned)(ntx * ntx), np);
    if (a.V2p > 0) {
      if (!a.pos)
        k_mp_xt<0><<<gx, 256, 0, s>>>(a.plist, p0, Vrp, a.m2pmax, a.m2, a.gV, a.b2off, a.BG2, ldd,
                                      a.d2pstride, a.D2t, a.d2tld, a.R, a.XT, cs);
      else if (bglabel)
        k_mp_xt<2><<<gx, 256, 0, s>>>(a.plist, p0, Vrp, a.m2pmax, a.m2, a.gV, a.b2off, a.BG2, ldd,
                                      a.d2pstride, a.D2t, a.d2tld, a.R, a.XT, cs);
      else
        k_mp_xt<1><<<gx, 256, 0, s>>>(a.plist, p0, Vrp, a.m2pmax, a.m2, a.gV, a.b2off, a.BG2, ldd,
                                      a.d2pstride, a.D2t, a.d2tld, a.R, a.XT, cs);
    }
    if (a.evt) {
      hipError_t e = hipEventRecord(a.evt[2 * c], s);
      if (e != hipSuccess) return e;
    }
    if (bglabel)
      k_mp_y<true><<<gy, 256, 0, s>>>(a.plist, p0, Vrp, a.m2pmax, a.m2, a.gV, a.XT, a.R, cs);
    else
      k_mp_y<false><<<gy, 256, 0, s>>>(a.plist, p0, Vrp, a.m2pmax, a.m2, a.gV, a.XT, a.R, cs);
    if (a.evt) {
      hipError_t e = hipEventRecord(a.evt[2 * c + 1], s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t launch_hier_level2_compose(const HierArgs& a, hipStream_t s) {
  return compose_level2(a, a.bglabel, a.cert_bad, a.cert_mbg, s);
}

hipError_t launch_flat_store(int32_t V, int64_t Vp, const u32* BG, const int32_t* bgcomp,
                             const int32_t* bgoff, const int32_t* nb, const int32_t* grp,
                             const int32_t* gbg0, int32_t* bgrow, int32_t* bgnb, int32_t* bggrp,
                             const int32_t* bglocal, u32* H, hipStream_t s) {
  if (V <= 0) return hipSuccess;
  k_hier_vmeta<<<hblocks(V), 256, 0, s>>>(V, bgcomp, bgoff, nb, grp, gbg0, bgrow, bgnb, bggrp);
  k_flat_store<<<(unsigned)V, 256, 0, s>>>(V, Vp, BG, bgrow, bgnb, bglocal, H);
  return hipGetLastError();
}

hipError_t launch_level3_a(const L3Args& a, hipStream_t s) {
  k_l3_gather<<<dim3((unsigned)a.V3gp, (unsigned)a.nT), 256, 0, s>>>(a.V2p, a.BG2, a.tbase, a.tsize,
                                                                      a.V3gp, a.M3);
  const int ntt = a.V3gp / 128;
  hipError_t e = (a.side && ntt > 1)
                     ? launch_dense_fw_batch_lookahead(a.M3, a.V3gp, 128, ntt, a.nT,
                                                       (int64_t)a.V3gp * a.V3gp, s, a.side, a.sync,
                                                       nullptr, a.kc, a.pivot)
                     : launch_dense_fw_batch(a.M3, a.V3gp, 128, ntt, a.nT, (int64_t)a.V3gp * a.V3gp,
                                             s, nullptr, a.kc, a.pivot);
  if (e != hipSuccess) return e;
  if (a.m > 0)
    k_l3_edges<<<hblocks(a.m), 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.comp, a.local, a.bgoff, a.grp,
                                            a.gpt, a.b2off, a.b2rank, a.flag3, nullptr, nullptr, 0,
                                            nullptr);
  k_b2_scan<<<(unsigned)a.nT, 256, 0, s>>>(a.tbase, a.tsize, a.flag3, a.V3gp, a.b3list, a.b3rank, a.m3);
  return hipGetLastError();
}

hipError_t launch_level3_b(const L3Args& a, hipStream_t s) {
  if (a.pos3) {  // the super-groups' positions and R_T by position
    k_pos_build<<<(unsigned)a.nT, 256, 0, s>>>(a.tbase, a.tsize, a.b3rank, a.b3list, a.m3, a.V3gp,
                                               a.V3rp, a.pos3);
    k_rpos_gather<<<dim3((unsigned)a.m3pmax, (unsigned)a.nT), 256, 0, s>>>(
        a.V3gp, a.V3rp, a.m3pmax, a.m3, a.b3list, a.pos3, a.M3, a.R3);
  } else {
    k_r_gather<<<dim3((unsigned)a.m3pmax, (unsigned)a.nT), 256, 0, s>>>(a.V3gp, a.m3pmax, a.m3,
                                                                         a.b3list, a.M3, a.R3);
  }
  if (a.V3p > 0) {
    k_bg2_init<<<(unsigned)a.V3p, 256, 0, s>>>(a.V3, a.V3p, a.nT, a.b3off, a.b3list, a.V3gp, a.M3,
                                               a.BG3);
    if (a.m > 0)
      k_l3_edges<<<hblocks(a.m), 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.comp, a.local, a.bgoff, a.grp,
                                              a.gpt, a.b2off, a.b2rank, nullptr, a.b3off, a.b3rank,
                                              a.V3p, a.BG3);
    const int nt = (int)(a.V3p / 128);
    hipError_t e = (a.side && nt > 1)
                       ? launch_dense_fw_lookahead(a.BG3, a.V3p, 128, nt, s, a.side, a.sync, nullptr,
                                                   a.kc, a.pivot)
                       : launch_dense_fw(a.BG3, a.V3p, 128, nt, s, nullptr, a.kc, a.pivot);
    if (e != hipSuccess) return e;
  }
  return launch_level3_compose(a, s);
}

hipError_t launch_level3_compose(const L3Args& a, hipStream_t s) {
  // with positions (the build): the first product copies T1's B3 positions
  // (the grid's second half) and stores the B3 columns of T2 into BG2, the
  // second runs over T2's other vertices; without (the test hook): plain
  const int32_t Vrp = a.pos3 ? a.V3rp : a.V3gp;
  const int ntx = Vrp / 128, ntm = a.m3pmax / 128;
  CompStore cs{};
  if (a.pos3) {
    cs.pos = a.pos3; cs.Vgp = a.V3gp; cs.ngroups = a.nT; cs.b2list = a.b3list; cs.Mg = a.M3;
    cs.dense = a.BG2; cs.ldo = a.V2p; cs.dbase = a.tbase;
  }
  for (int32_t p0 = 0; p0 < a.npairs; p0 += a.chunk) {
    const unsigned np = (unsigned)min(a.chunk, a.npairs - p0);
    if (a.V3p > 0) {
      const dim3 gx((unsigned)(ntm * ntx * (a.pos3 ? 2 : 1)), np);
      if (a.pos3)
        k_mp_xt<1><<<gx, 256, 0, s>>>(a.plist, p0, Vrp, a.m3pmax, a.m3, a.tsize, a.b3off, a.BG3, a.V3p, 0,
                                      nullptr, 0, a.R3, a.XT3, cs);
      else
        k_mp_xt<0><<<gx, 256, 0, s>>>(a.plist, p0, Vrp, a.m3pmax, a.m3, a.tsize, a.b3off, a.BG3, a.V3p, 0,
                                      nullptr, 0, a.R3, a.XT3, cs);
    }
    k_mp_y_dense<<<dim3((unsigned)(ntx * ntx), np), 256, 0, s>>>(
        a.plist, p0, a.V3gp, Vrp, a.m3pmax, a.m3, a.tsize, a.tbase, a.pos3, a.XT3, a.R3, a.M3, a.BG2,
        a.V2p);
  }
  return hipGetLastError();
}

hipError_t launch_hier_row(const HierArgs& a, int32_t x, u32* out, hipStream_t s) {
  k_hier_row<<<(unsigned)((a.V + 255) / 256 > 0 ? (a.V + 255) / 256 : 1), 256, 0, s>>>(
      x, a.share_groups > 0 ? 0 : 1, a.V, a.ngroups, a.bggrp, a.bgrow, a.bgnb, a.bglocal, a.gV,
      a.pairbase, a.H, out);
  return hipGetLastError();
}

}  // namespace spq

namespace spq {

hipError_t launch_share_prepare(const HierArgs& a, const ShareBlocks& b, hipStream_t s) {
  launch_rpos(a, s);
  k_blk_init<<<dim3((unsigned)b.bpmax, (unsigned)b.nblk), 256, 0, s>>>(a.Vgp, b.bpmax, b.bfirst,
                                                                       a.b2off, a.b2list, a.Mg,
                                                                       b.A);
  if (b.multi) {
    if (a.m > 0)
      k_blk_edges<<<hblocks(a.m), 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.comp, a.local, a.bgoff, a.grp,
                                               b.gblk, b.bfirst, a.b2off, a.b2rank, b.bpmax, b.A);
    hipError_t e = launch_dense_fw_batch(b.A, b.bpmax, 128, b.bpmax / 128, b.nblk,
                                         (int64_t)b.bpmax * b.bpmax, s, nullptr, a.kc, a.pivot);
    if (e != hipSuccess) return e;
  }
  k_dt_init<<<(unsigned)a.V2p, 256, 0, s>>>(a.V2, a.S2, a.S2p, b.nblk, b.boff, b.bpmax, b.A, a.DT);
  if (a.m > 0)
    k_cross_collect<<<hblocks(a.m), 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.comp, a.local, a.bgoff, a.grp,
                                                 b.gblk, a.b2off, a.b2rank, a.xcount, a.xe);
  return hipGetLastError();
}

hipError_t launch_share_b3_lists(const HierArgs& a, const ShareBlocks& b, uint8_t* flag3,
                                 uint8_t* flagn, int32_t* b3list, int32_t* nb3list, int32_t* b3rank,
                                 int32_t* nrank, int32_t* m3, int32_t* n3, hipStream_t s) {
  hipError_t e = hipMemsetAsync(flag3, 0, (size_t)(a.V2 > 0 ? a.V2 : 1), s);
  if (e != hipSuccess) return e;
  if (a.m > 0) k_b3_mark<<<hblocks(2 * a.m), 256, 0, s>>>(a.xcount, a.xe, flag3);
  if (a.V2 > 0) k_flag_not<<<hblocks(a.V2), 256, 0, s>>>(a.V2, flag3, flagn);
  k_b2_scan<<<(unsigned)b.nblk, 256, 0, s>>>(b.boff, b.bsize, flag3, b.bpmax, b3list, b3rank, m3);
  k_b2_scan<<<(unsigned)b.nblk, 256, 0, s>>>(b.boff, b.bsize, flagn, b.bpmax, nb3list, nrank, n3);
  return hipGetLastError();
}

hipError_t launch_share_b3_gather(const ShareBlocks& b, const ShareB3& c, hipStream_t s) {
  k_a3_gather<<<dim3((unsigned)c.b3pmax, (unsigned)b.nblk), 256, 0, s>>>(b.bpmax, c.b3pmax, c.m3,
                                                                          c.b3list, b.A, c.A3);
  k_aout_gather<<<dim3((unsigned)c.b3pmax, (unsigned)b.nblk), 256, 0, s>>>(
      b.bpmax, c.b3pmax, c.n3pmax, c.m3, c.n3, c.b3list, c.nb3list, b.A, c.Aout);
  return hipGetLastError();
}

// One Bellman-Ford round, in place on DT: intra-block step on the B3 rows,
// then cross edges.
hipError_t launch_share_round(const HierArgs& a, const ShareBlocks& b, const ShareB3& c, int32_t nxe,
                              const BfRound& r, hipStream_t s) {
  const int ntm = c.b3pmax / 128, ntc = (int)(a.S2p / 128);
  k_bf_intra3<<<dim3((unsigned)(ntm * ntc), (unsigned)b.nblk), 256, 0, s>>>(
      b.bpmax, c.b3pmax, a.S2p, c.m3, b.boff, c.b3list, c.A3, a.DT, r.dirty, r.cnt, r.list);
  if (nxe > 0)
    k_bf_cross<<<(unsigned)nxe, 256, 0, s>>>(nxe, a.xe, a.S2, a.S2p, a.DT, r.dirty, r.dirty_next,
                                             c.b3rank, c.b3pmax, r.round, r.stamp, r.cnt_next,
                                             r.list_next);
  return hipGetLastError();
}

hipError_t launch_share_final(const HierArgs& a, const ShareBlocks& b, const ShareB3& c,
                              hipStream_t s) {
  const int ntm = c.n3pmax / 128, ntc = (int)(a.S2p / 128);
  k_bf_final<<<dim3((unsigned)(ntm * ntc), (unsigned)b.nblk), 256, 0, s>>>(
      b.bpmax, c.b3pmax, c.n3pmax, a.S2p, c.m3, c.n3, b.boff, c.b3list, c.nb3list, c.Aout, a.DT);
  return hipGetLastError();
}

hipError_t launch_bf_rows(int32_t ngroups, int32_t lstride, int32_t kp, int64_t ldc,
                          const int32_t* nk, const int32_t* zero, const int32_t* own, const u32* A,
                          u32* C, const u32* dirty, const int32_t* rcnt, const int32_t* rlist,
                          hipStream_t s) {
  const int ntm = kp / 128, ntc = (int)(ldc / 128);
  k_bf_intra3<<<dim3((unsigned)(ntm * ntc), (unsigned)ngroups), 256, 0, s>>>(
      lstride, kp, ldc, nk, zero, own, A, C, dirty, rcnt, rlist);
  return hipGetLastError();
}

hipError_t launch_bf_gather(int32_t ngroups, int32_t lstride, int32_t kp, int32_t np, int64_t ldc,
                            const int32_t* nk, const int32_t* nout, const int32_t* zero,
                            const int32_t* own, const int32_t* out, const u32* Aout, u32* C,
                            hipStream_t s) {
  const int ntm = np / 128, ntc = (int)(ldc / 128);
  k_bf_final<<<dim3((unsigned)(ntm * ntc), (unsigned)ngroups), 256, 0, s>>>(
      lstride, kp, np, ldc, nk, nout, zero, own, out, Aout, C);
  return hipGetLastError();
}

hipError_t launch_share_compose(const HierArgs& a, const u32* DT, hipStream_t s) {
  dim3 tg((unsigned)((a.S2p + 31) / 32), (unsigned)(a.m2pmax / 32), (unsigned)a.ngroups);
  k_panel_transpose<<<tg, 256, 0, s>>>(DT, a.S2p, a.m2pmax, a.m2, a.b2off, a.BG2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  HierArgs p = a;
  p.d2ld = a.m2pmax;
  p.d2pstride = a.S2p * a.m2pmax;
  return compose_level2(p, nullptr, nullptr, nullptr, s);
}

}  // namespace spq
