// HIP kernels of the shortest-path query structure (gfx950).
//
// Steps, in the order the build runs them:
//   partition  k_count_part, k_edges_scan, k_count_boundary, k_members, k_rank
//              (boundary detection and the Fig. 1 renumbering, Sections 2, 4)
//   APSP(C)    k_comp_init, k_comp_edges, k_comp_fw (Algorithm 1, Phase 2)
//   BG         k_bg_init, k_bg_edges (Algorithm 1, Phase 2 clique edges and
//              Phase 3 boundary graph); its all-pairs distances are the
//              blocked Floyd-Warshall of fw.hip
//   query      k_query (Algorithm 2)
#include "spq_internal.h"
#include "tiles.h"

namespace spq {

// ------------------------------------------------------------ partition ---
__global__ void k_count_part(int32_t n, const int32_t* __restrict__ part, int32_t k,
                             int32_t* __restrict__ cnt, u32* __restrict__ err) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t p = part[v];
  if (p < 0 || p >= k) {
    atomicOr(err, ERR_PART);
    return;
  }
  atomicAdd(&cnt[p], 1);
}

// Validates the edges, marks the boundary (Section 2: a vertex with a
// neighbour in another component) and sums the weights: per component for
// edges inside it, and in total.
__global__ void k_edges_scan(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                             const int32_t* __restrict__ w, int32_t n, const int32_t* __restrict__ part,
                             int32_t k, uint8_t* __restrict__ flag, unsigned long long* __restrict__ sumc,
                             unsigned long long* __restrict__ total, u32* __restrict__ err) {
  unsigned long long acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = eu[e], v = ev[e], x = w[e];
    if (u < 0 || u >= n || v < 0 || v >= n) {
      atomicOr(err, ERR_VERTEX);
      continue;
    }
    if (x < 0 || (u32)x >= INF) {
      atomicOr(err, ERR_WEIGHT);
      continue;
    }
    int32_t pu = part[u], pv = part[v];
    if (pu < 0 || pu >= k || pv < 0 || pv >= k) continue;  // reported by k_count_part
    if (pu != pv) {
      flag[u] = 1;
      flag[v] = 1;
    } else if (u != v) {
      atomicAdd(&sumc[pu], (unsigned long long)x);
    }
    acc += (unsigned long long)x;
  }
  // wave reduction, then one atomic per wave
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0 && acc) atomicAdd(total, acc);
}

__global__ void k_count_boundary(int32_t n, const int32_t* __restrict__ part,
                                 const uint8_t* __restrict__ flag, int32_t* __restrict__ nb) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (flag[v]) atomicAdd(&nb[part[v]], 1);
}

// Groups the vertices by component (arbitrary order inside a component); the
// boundary flag rides in bit 31.
__global__ void k_members(int32_t n, const int32_t* __restrict__ part, const uint8_t* __restrict__ flag,
                          const int32_t* __restrict__ off, int32_t* __restrict__ fill,
                          u32* __restrict__ members) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t c = part[v];
  int32_t slot = atomicAdd(&fill[c], 1);
  members[off[c] + slot] = (u32)v | ((u32)flag[v] << 31);
}

// Renumbering (Section 4, Fig. 1): inside each component the boundary vertices
// come first, each group in ascending vertex id.  The rank of a vertex is the
// number of members of its component with the same flag and a smaller id.
__global__ void k_rank(int32_t n, int32_t k, const u32* __restrict__ members,
                       const int32_t* __restrict__ off, const int32_t* __restrict__ nb,
                       const int32_t* __restrict__ bgoff, int32_t* __restrict__ comp,
                       int32_t* __restrict__ local, int32_t* __restrict__ bgcomp,
                       int32_t* __restrict__ bglocal, int32_t* __restrict__ bgvert) {
  int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= n) return;
  // component of this position: largest c with off[c] <= pos
  int32_t lo = 0, hi = k - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= pos) lo = mid; else hi = mid - 1;
  }
  const int32_t c = lo;
  const u32 me = members[pos];
  const u32 id = me & 0x7fffffffu, f = me >> 31;
  int32_t rank = 0;
  for (int32_t x = off[c]; x < off[c + 1]; x++) {
    u32 o = members[x];
    rank += ((o >> 31) == f) & ((o & 0x7fffffffu) < id);
  }
  int32_t l = f ? rank : nb[c] + rank;
  comp[id] = c;
  local[id] = l;
  if (f) {
    bgcomp[bgoff[c] + l] = c;
    bglocal[bgoff[c] + l] = l;
    bgvert[bgoff[c] + l] = (int32_t)id;
  }
}

// --------------------------------------------------------------- APSP(C) --
// Component matrices are P x P (P = |C| rounded up to 64), row-major at
// element moff[c].  Initial value (Section 4): 0 on the diagonal, INF
// elsewhere; edges are scattered next.  Padding rows/columns stay isolated.
__global__ void k_comp_init(const int32_t* __restrict__ P, const int64_t* __restrict__ moff,
                            u32* __restrict__ M) {
  const int32_t c = blockIdx.x;
  const int32_t p = P[c];
  u32* base = M + moff[c];
  const int64_t quads = (int64_t)p * p / 4;
  for (int64_t q = threadIdx.x; q < quads; q += blockDim.x) {
    int64_t e = q * 4;
    int32_t i = (int32_t)(e / p), j = (int32_t)(e % p);
    uint4 v = make_uint4(INF, INF, INF, INF);
    if (i >= j && i < j + 4) {
      if (i == j) v.x = 0;
      if (i == j + 1) v.y = 0;
      if (i == j + 2) v.z = 0;
      if (i == j + 3) v.w = 0;
    }
    reinterpret_cast<uint4*>(base)[q] = v;
  }
}

// Edges inside a component become matrix entries; parallel edges keep the
// lightest one, self-loops are dropped.
__global__ void k_comp_edges(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                             const int32_t* __restrict__ w, const int32_t* __restrict__ comp,
                             const int32_t* __restrict__ local, const int32_t* __restrict__ P,
                             const int64_t* __restrict__ moff, u32* __restrict__ M) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = eu[e], v = ev[e];
    if (u == v) continue;
    int32_t c = comp[u];
    if (c != comp[v]) continue;
    int64_t p = P[c];
    u32* base = M + moff[c];
    int32_t lu = local[u], lv = local[v];
    atomicMin(base + lu * p + lv, (u32)w[e]);
    atomicMin(base + lv * p + lu, (u32)w[e]);
  }
}

// Phase 2: one workgroup closes one whole component matrix by blocked
// Floyd-Warshall with 64 x 64 tiles (diagonal tile, then its row - written
// twice, once transposed as the column - then all other tiles).  The matrix
// stays in global memory between the tile steps; it is a few hundred KB at
// most and stays in L2.  order[] lists components largest first.
__global__ __launch_bounds__(256) void k_comp_fw(const int32_t* __restrict__ order,
                                                 const int32_t* __restrict__ P,
                                                 const int64_t* __restrict__ moff, u32* M) {
  constexpr int T = 64;
  __shared__ __attribute__((aligned(16))) u32 sA[T * T];
  __shared__ __attribute__((aligned(16))) u32 sB[T * T];
  __shared__ __attribute__((aligned(16))) u32 rb[4 * T];
  const int32_t c = order[blockIdx.x];
  const int64_t p = P[c];
  const int nt = (int)(p / T);
  u32* base = M + moff[c];
  u32 t[T / 16][T / 16];
  for (int r = 0; r < nt; r++) {
    u32* D = base + (int64_t)r * T * p + r * T;
    tile_load<T>(t, D, p);
    fw_tile<T>(t, rb);
    tile_store<T>(t, D, p);
    if (nt == 1) break;
    tile_to_lds<T>(t, sA);
    __syncthreads();
    // row r and (by symmetry) column r of tiles
    for (int j = 0; j < nt; j++) {
      if (j == r) continue;
      u32* Rj = base + (int64_t)r * T * p + j * T;
      tile_load<T>(t, Rj, p);
      tile_to_lds<T>(t, sB);
      __syncthreads();
      minplus_lds<T>(t, sA, sB, T);
      tile_store<T>(t, Rj, p);
      tile_store_t<T>(t, base + (int64_t)j * T * p + r * T, p);
      __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    // the remaining tiles: T(i,j) = min(T(i,j), T(i,r) (x) T(r,j)), with
    // T(i,r)^T = T(r,i) already laid out as the transposed left operand;
    // only i <= j is computed, T(j,i) receives the transpose
    for (int i = 0; i < nt; i++) {
      if (i == r) continue;
      tile_load<T>(t, base + (int64_t)r * T * p + i * T, p);
      tile_to_lds<T>(t, sA);
      for (int j = i; j < nt; j++) {
        if (j == r) continue;
        tile_load<T>(t, base + (int64_t)r * T * p + j * T, p);
        tile_to_lds<T>(t, sB);
        u32* Cij = base + (int64_t)i * T * p + j * T;
        tile_load<T>(t, Cij, p);
        __syncthreads();
        minplus_lds<T>(t, sA, sB, T);
        tile_store<T>(t, Cij, p);
        if (j != i) tile_store_t<T>(t, base + (int64_t)j * T * p + i * T, p);
        __syncthreads();
      }
    }
    __threadfence_block();
    __syncthreads();
  }
}

// -------------------------------------------------------------------- BG --
// BG matrix, Vp x Vp (Vp = V rounded up to the tile): within one component
// the APSP(C) distance between its boundary vertices (the clique edges of
// Algorithm 1; they are never heavier than a G edge between the same pair),
// 0 on the diagonal, INF elsewhere and on the padding.
__global__ void k_bg_init(int32_t V, int64_t Vp, const int32_t* __restrict__ bgcomp,
                          const int32_t* __restrict__ bglocal, const int32_t* __restrict__ nb,
                          const int32_t* __restrict__ bgoff, const int32_t* __restrict__ P,
                          const int64_t* __restrict__ moff, const u32* __restrict__ M,
                          u32* __restrict__ BG) {
  const int64_t row = blockIdx.x;
  u32* out = BG + row * Vp;
  // BG ids are grouped by component, so the row's own component is the
  // column range [lo, hi)
  int64_t lo = 0, hi = 0;
  const u32* mrow = nullptr;
  if (row < V) {
    const int32_t cr = bgcomp[row];
    lo = bgoff[cr];
    hi = lo + nb[cr];
    mrow = M + moff[cr] + (int64_t)bglocal[row] * P[cr] - lo;
  }
  for (int64_t q0 = (int64_t)threadIdx.x * 4; q0 < Vp; q0 += (int64_t)blockDim.x * 4) {
    u32 v[4];
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const int64_t q = q0 + s;
      v[s] = (q == row) ? 0u : (q >= lo && q < hi) ? mrow[q] : INF;
    }
    *reinterpret_cast<uint4*>(out + q0) = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

// Edges of G between boundary vertices of different components.
__global__ void k_bg_edges(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                           const int32_t* __restrict__ w, const int32_t* __restrict__ comp,
                           const int32_t* __restrict__ local, const int32_t* __restrict__ bgoff,
                           int64_t Vp, u32* __restrict__ BG) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = eu[e], v = ev[e];
    int32_t cu = comp[u], cv = comp[v];
    if (cu == cv) continue;
    int64_t a = bgoff[cu] + local[u], b = bgoff[cv] + local[v];
    atomicMin(BG + a * Vp + b, (u32)w[e]);
    atomicMin(BG + b * Vp + a, (u32)w[e]);
  }
}

// ----------------------------------------------------------------- query --
// Per-vertex query record (layout in spq_internal.h): where the vertex's row
// of APSP(C) starts, its component and local index, its component's |B(C)|
// and place in its group, and its group's size and band in the blocked store,
// so a query needs no other table.
__global__ void k_vrec(int32_t n, const int32_t* __restrict__ comp, const int32_t* __restrict__ local,
                       const int64_t* __restrict__ moff, const int32_t* __restrict__ P,
                       const int32_t* __restrict__ bgoff, const int32_t* __restrict__ nb,
                       const int32_t* __restrict__ grp, const int32_t* __restrict__ gbg0,
                       const int32_t* __restrict__ gV, const int64_t* __restrict__ gT,
                       u32* __restrict__ vrec) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t c = comp[v], l = local[v], s = grp[c];
  const uint64_t row = (uint64_t)(moff[c] + (int64_t)l * P[c]);
  const uint64_t t = (uint64_t)gT[s];
  uint4* r = reinterpret_cast<uint4*>(vrec + v * VREC_WORDS);
  r[0] = make_uint4((u32)row, (u32)(row >> 32), (u32)c, (u32)l);
  r[1] = make_uint4((u32)gbg0[s], (u32)nb[c], (u32)s, (u32)(bgoff[c] - gbg0[s]));
  r[2] = make_uint4((u32)gV[s], 0u, (u32)t, (u32)(t >> 32));
}

// Algorithm 2, one query at a time per half-wave (32 lanes, 8 per workgroup):
//   t(b2) = min over b1 of dist_C1(v1, b1) + dist_BG(b1, b2)     (first stage)
//   r     = min over b2 of t(b2) + dist_C2(b2, v2)                (second stage)
//   r     = min(r, dist_C1(v1, v2)) if C1 = C2                    (same component)
// The B(C1) x B(C2) block of BG distances is read row by row in uint4
// pieces: L = ceil(columns / 4) lanes per row, R = 32 / L rows per load, and
// QU loads in flight per lane, each with its dist_C1(v1, b1) (the prefix of
// v1's row of APSP(C1), boundary first).  A lane keeps the first-stage
// minimum of its four columns over its rows and adds dist_C2(b2, v2) (v2's
// row, the matrix being symmetric); the half-wave then takes the minimum.
// The blocked BG store keeps each B(C1) x B(C2) block as one contiguous run
// (rows |B(C2)| apart).  Block columns come in chunks of 128 when
// |B(C2)| > 128.
// The two vertex records (24 words) are spread one word per lane over lanes
// 0-23 and read with ds_bpermute; they locate the block without any other
// table.
#ifndef SPQ_QUERY_UNROLL
#define SPQ_QUERY_UNROLL 6
#endif

__device__ __forceinline__ uint4 load4_upto(const u32* p, int valid) {
  if (valid >= 4) return *reinterpret_cast<const uint4*>(p);
  return make_uint4(valid > 0 ? p[0] : INF, valid > 1 ? p[1] : INF, valid > 2 ? p[2] : INF, INF);
}

__device__ __forceinline__ u32 hw_word(u32 x, int lane) { return (u32)__shfl((int)x, lane, 32); }

// ids (lanes 0, 1) of pair i, or 0 past the end
__device__ __forceinline__ u32 load_ids(int64_t i, int64_t q, const int32_t* v1, const int32_t* v2,
                                        int l) {
  if (i >= q || l > 1) return 0u;
  return (u32)(l == 0 ? v1[i] : v2[i]);
}

// records of both endpoints (lanes 0-23), if both ids are valid
__device__ __forceinline__ u32 load_recs(u32 ids, int32_t n, const u32* vrec, int l, bool& ok) {
  const int32_t a = (int32_t)hw_word(ids, 0), b = (int32_t)hw_word(ids, 1);
  ok = a >= 0 && a < n && b >= 0 && b < n;
  if (!ok || l >= 2 * VREC_WORDS) return 0u;
  const int32_t v = l < VREC_WORDS ? a : b;
  return vrec[(int64_t)v * VREC_WORDS + (l < VREC_WORDS ? l : l - VREC_WORDS)];
}

// dist(v1, v2) by one half-wave from the two records spread over lanes 0-23
// (load_recs); every lane of the half-wave calls it with the same records and
// gets the result.  0xffffffff (SPQ_BAD_PAIR) when v1 lies outside a share.
__device__ __forceinline__ u32 hw_pair_dist(u32 rec, int l, const u32* __restrict__ M,
                                            const u32* __restrict__ H, int32_t share_comps) {
  constexpr int QU = SPQ_QUERY_UNROLL;
  if (share_comps > 0 && (int32_t)hw_word(rec, 2) >= share_comps) return 0xffffffffu;
  // the full two-level store keeps group pairs S1 <= S2 only; dist is
  // symmetric, so take the endpoints in group order when needed (a share
  // keeps all S2): words o1 + j describe the first, o2 + j the second
  const bool sw = share_comps == 0 && hw_word(rec, 6) > hw_word(rec, VREC_WORDS + 6);
  const int o1 = sw ? VREC_WORDS : 0, o2 = sw ? 0 : VREC_WORDS;
  const u32* row1 = M + ((uint64_t)hw_word(rec, o1) | ((uint64_t)hw_word(rec, o1 + 1) << 32));
  const u32* row2 = M + ((uint64_t)hw_word(rec, o2) | ((uint64_t)hw_word(rec, o2 + 1) << 32));
  const int32_t nb1 = (int32_t)hw_word(rec, o1 + 5), nb2 = (int32_t)hw_word(rec, o2 + 5);
  // band of group S1, then the pair block: S1's rows against the groups
  // before S2 in the band (from S1 itself in the full store)
  const int64_t band = (int64_t)((uint64_t)hw_word(rec, o1 + 10) |
                                 ((uint64_t)hw_word(rec, o1 + 11) << 32));
  const int64_t gv1 = hw_word(rec, o1 + 8);
  const int64_t pb = band + gv1 * ((int64_t)hw_word(rec, o2 + 4) -
                                   (share_comps ? 0 : (int64_t)hw_word(rec, o1 + 4)));
  const u32* blk = H + pb + (int64_t)hw_word(rec, o1 + 7) * hw_word(rec, o2 + 8) +
                   (int64_t)nb1 * hw_word(rec, o2 + 7);
  const int64_t ld = nb2;
  const bool same = hw_word(rec, 2) == hw_word(rec, VREC_WORDS + 2);
  const u32 loc2 = hw_word(rec, o2 + 3);
  u32 best = INF;
  for (int32_t c0 = 0; c0 < nb2; c0 += 128) {
    const int32_t nbc = min(128, nb2 - c0);
    const int L = (nbc + 3) >> 2, R = 32 / L;
    const int r = l / L, col = c0 + (l - r * L) * 4;
    const bool lane_on = r < R;
    const int cvalid = c0 + nbc - col;  // columns of this lane's piece (>= 1 when on)
    // second-stage terms first: independent of the block
    u32 e[4];
#pragma unroll
    for (int j = 0; j < 4; j++) e[j] = (lane_on && j < cvalid) ? row2[col + j] : INF;
    u32 t[4] = {INF, INF, INF, INF};
    for (int32_t r0 = 0; r0 < nb1; r0 += R * QU) {
      uint4 v[QU];
      u32 d[QU];
#pragma unroll
      for (int u = 0; u < QU; u++) {
        const int32_t row = r0 + u * R + r;
        const bool on = lane_on && row < nb1;
        v[u] = on ? load4_upto(blk + (int64_t)row * ld + col, cvalid) : make_uint4(INF, INF, INF, INF);
        d[u] = on ? row1[row] : INF;
      }
#pragma unroll
      for (int u = 0; u < QU; u++) {
        t[0] = min(t[0], d[u] + v[u].x);
        t[1] = min(t[1], d[u] + v[u].y);
        t[2] = min(t[2], d[u] + v[u].z);
        t[3] = min(t[3], d[u] + v[u].w);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; j++) best = min(best, min(t[j], INF) + e[j]);
  }
  for (int o = 16; o > 0; o >>= 1) best = min(best, (u32)__shfl_xor((int)best, o));
  if (same) best = min(best, row1[loc2]);
  return min(best, INF);
}

// 64 VGPRs: eight waves per SIMD keep enough block loads in flight
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_query(
    int64_t q, const int32_t* __restrict__ v1, const int32_t* __restrict__ v2,
    int32_t* __restrict__ out, int32_t n, const u32* __restrict__ vrec, const u32* __restrict__ M,
    const u32* __restrict__ H, int32_t share_comps) {
  const int64_t qi = (int64_t)blockIdx.x * 8 + (threadIdx.x >> 5);
  const int l = threadIdx.x & 31;
  if (qi >= q) return;  // whole half-waves only
  bool ok;
  const u32 rec = load_recs(load_ids(qi, q, v1, v2, l), n, vrec, l, ok);
  const u32 res = ok ? hw_pair_dist(rec, l, M, H, share_comps) : 0xffffffffu;  // SPQ_BAD_PAIR
  if (l == 0) out[qi] = (int32_t)res;
}

// ------------------------------------------------------------------ paths --
// One shortest path per half-wave, walked back from t to s on the graph's
// adjacency: at vertex c (dist(s, c) = D), any neighbour u over an edge of
// weight w with dist(s, u) + w = D lies on a shortest s-c path, so the walk
// steps to it, preferring dist(s, u) < D; every dist(s, u) is an Algorithm 2
// query on the index.  With positive weights dist falls at every step and the
// walk reaches s.  A zero-weight edge allows a step at equal distance; such a
// step avoids the last 8 vertices of the walk and its last 16 dead ends, and
// a vertex with no step at all is a dead end the walk backs out of.  A walk
// that backs out past t, or runs 4 max_len + 1,024 steps, is reported (-3).
// Lane 0 writes the vertices (t first) and reverses them at the end, so the
// path reads s .. t.
//   lens[i]: vertices on the path (>= 1), 0 no path, -1 bad pair (an id
//   outside [0, n), or v1 outside a share), -2 the walk needed more than
//   max_len vertices, -3 it found no way off a zero-weight plateau
__device__ __forceinline__ u32 hw_dist_to(int32_t s, int32_t u, int32_t n, const u32* vrec,
                                          const u32* M, const u32* H, int32_t share_comps, int l) {
  bool ok;
  const u32 ids = l == 0 ? (u32)s : (l == 1 ? (u32)u : 0u);
  const u32 rec = load_recs(ids, n, vrec, l, ok);
  return ok ? hw_pair_dist(rec, l, M, H, share_comps) : 0xffffffffu;
}

__global__ __launch_bounds__(256) void k_paths(
    int64_t q, const int32_t* __restrict__ v1, const int32_t* __restrict__ v2, int32_t max_len,
    int32_t n, const u32* __restrict__ vrec, const u32* __restrict__ M, const u32* __restrict__ H,
    int32_t share_comps, const int64_t* __restrict__ rowptr, const int2* __restrict__ adj,
    const int32_t* __restrict__ wts, int32_t* __restrict__ paths, int32_t* __restrict__ lens) {
  const int64_t qi = (int64_t)blockIdx.x * 8 + (threadIdx.x >> 5);
  const int l = threadIdx.x & 31;
  if (qi >= q) return;  // whole half-waves only
  const int32_t s = v1[qi], t = v2[qi];
  int32_t* out = paths + qi * (int64_t)max_len;
  int32_t code = 0;
  u32 dcur = 0xffffffffu;
  if (s >= 0 && s < n && t >= 0 && t < n) dcur = hw_dist_to(s, t, n, vrec, M, H, share_comps, l);
  if (dcur == 0xffffffffu) code = -1;
  int32_t len = 0;
  if (code == 0 && dcur < INF) {
    // lanes 0-7: the vertices at path positions p (slot p mod 8) of the last
    // 8 pushed; lanes 0-15: the last 16 dead ends
    int32_t cur = t, recent = l == 0 ? t : -1, dead = -1, ndead = 0;
    if (l == 0) out[0] = t;
    len = 1;
    const int64_t iter_cap = 4 * (int64_t)max_len + 1024;
    for (int64_t iter = 0; cur != s; iter++) {
      if (iter > iter_cap) {
        code = -3;
        break;
      }
      int32_t next = -1;
      u32 dnext = INF;
      const int64_t e1 = rowptr[cur + 1];
      for (int64_t e = rowptr[cur]; e < e1; e++) {
        const int2 a = adj[e];
        const u32 w = (u32)wts[a.y];
        if (w > dcur || a.x == cur) continue;
        const u32 du = hw_dist_to(s, a.x, n, vrec, M, H, share_comps, l);
        if (du >= INF || du + w != dcur) continue;
        if (du < dcur) {
          next = a.x;
          dnext = du;
          break;
        }
        if (next < 0) {  // a zero-weight step: not to a recent vertex or a dead end
          const uint64_t seen = __ballot((l < 8 && recent == a.x) || (l < 16 && dead == a.x));
          if (((seen >> (threadIdx.x & 32)) & 0xffffu) == 0) {
            next = a.x;
            dnext = du;
          }
        }
      }
      if (next >= 0) {
        if (len >= max_len) {
          code = -2;
          break;
        }
        if (l == (len & 7)) recent = next;
        cur = next;
        dcur = dnext;
        if (l == 0) out[len] = cur;
        len++;
      } else {
        // a dead end (only on zero-weight plateaus): mark it, step back
        if (l == (ndead & 15)) dead = cur;
        ndead++;
        if (--len == 0) {
          code = -3;
          break;
        }
        int32_t prev = 0;
        if (l == 0) prev = out[len - 1];  // written by this lane
        cur = __shfl(prev, 0, 32);
        dcur = hw_dist_to(s, cur, n, vrec, M, H, share_comps, l);
      }
    }
  }
  if (l == 0) {
    if (code == 0 && len > 0) {
      for (int32_t i = 0, j = len - 1; i < j; i++, j--) {
        const int32_t x = out[i];
        out[i] = out[j];
        out[j] = x;
      }
      lens[qi] = len;
    } else {
      lens[qi] = code;
    }
  }
}

// Adjacency of G for the path walk: both directions of every edge that is not
// a self-loop, as (neighbour, edge index).
__global__ void k_adj_count(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            unsigned long long* __restrict__ deg) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = eu[e], v = ev[e];
    if (u == v) continue;
    atomicAdd(deg + u, 1ull);
    atomicAdd(deg + v, 1ull);
  }
}

// Exclusive prefix sum of deg[0, n) into rowptr[0, n] by one workgroup, in
// chunks of 1,024 (n is at most a few million: microseconds).
__global__ __launch_bounds__(256) void k_adj_scan(int32_t n, const unsigned long long* __restrict__ deg,
                                                  int64_t* __restrict__ rowptr) {
  __shared__ unsigned long long part[256];
  unsigned long long carry = 0;
  for (int64_t base = 0; base < n; base += 1024) {
    unsigned long long x[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t i = base + threadIdx.x * 4 + j;
      x[j] = i < n ? deg[i] : 0ull;
      sum += x[j];
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {  // inclusive scan of the 256 partial sums
      const unsigned long long y = threadIdx.x >= o ? part[threadIdx.x - o] : 0ull;
      __syncthreads();
      part[threadIdx.x] += y;
      __syncthreads();
    }
    unsigned long long run = carry + (threadIdx.x ? part[threadIdx.x - 1] : 0ull);
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t i = base + threadIdx.x * 4 + j;
      if (i < n) rowptr[i] = (int64_t)run;
      run += x[j];
    }
    carry += part[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) rowptr[n] = (int64_t)carry;
}

__global__ void k_adj_fill(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                           unsigned long long* __restrict__ cursor, int2* __restrict__ adj) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = eu[e], v = ev[e];
    if (u == v) continue;
    adj[atomicAdd(cursor + u, 1ull)] = make_int2(v, (int32_t)e);
    adj[atomicAdd(cursor + v, 1ull)] = make_int2(u, (int32_t)e);
  }
}

// ---------------------------------------------------------------- launch --
#define LAUNCH_CHECK() return hipGetLastError()

static inline unsigned blocks_for(int64_t items, int per = 256) {
  int64_t b = (items + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_partition_scan(const PartArgs& a, hipStream_t s) {
  if (a.n > 0) k_count_part<<<blocks_for(a.n), 256, 0, s>>>(a.n, a.part, a.k, a.cnt, a.err);
  if (a.m > 0) {
    unsigned g = blocks_for(a.m);
    if (g > 4096) g = 4096;
    k_edges_scan<<<g, 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.n, a.part, a.k, a.flag, a.sumc, a.total,
                                   a.err);
  }
  if (a.n > 0) k_count_boundary<<<blocks_for(a.n), 256, 0, s>>>(a.n, a.part, a.flag, a.nb);
  LAUNCH_CHECK();
}

hipError_t launch_edges_scan(const PartArgs& a, hipStream_t s) {
  if (a.m > 0) {
    unsigned g = blocks_for(a.m);
    if (g > 4096) g = 4096;
    k_edges_scan<<<g, 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.n, a.part, a.k, a.flag, a.sumc, a.total,
                                   a.err);
  }
  LAUNCH_CHECK();
}

hipError_t launch_renumber(const PartArgs& a, hipStream_t s) {
  k_members<<<blocks_for(a.n), 256, 0, s>>>(a.n, a.part, a.flag, a.off, a.fill, a.members);
  k_rank<<<blocks_for(a.n), 256, 0, s>>>(a.n, a.k, a.members, a.off, a.nb, a.bgoff, a.comp, a.local,
                                         a.bgcomp, a.bglocal, a.bgvert);
  k_vrec<<<blocks_for(a.n), 256, 0, s>>>(a.n, a.comp, a.local, a.moff, a.P, a.bgoff, a.nb, a.grp,
                                         a.gbg0, a.gV, a.gT, a.vrec);
  LAUNCH_CHECK();
}

hipError_t launch_components(const CompArgs& a, hipStream_t s) {
  k_comp_init<<<a.k, 256, 0, s>>>(a.P, a.moff, a.M);
  if (a.m > 0) {
    unsigned g = blocks_for(a.m);
    if (g > 8192) g = 8192;
    k_comp_edges<<<g, 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.comp, a.local, a.P, a.moff, a.M);
  }
  LAUNCH_CHECK();
}

hipError_t launch_comp_fw(int32_t count, const int32_t* order, const int32_t* P, const int64_t* moff,
                          u32* M, hipStream_t s) {
  if (count > 0) k_comp_fw<<<count, 256, 0, s>>>(order, P, moff, M);
  LAUNCH_CHECK();
}

hipError_t launch_bg_assembly(const BgArgs& a, hipStream_t s) {
  if (a.Vp == 0) return hipSuccess;
  k_bg_init<<<(unsigned)a.Vp, 256, 0, s>>>(a.V, a.Vp, a.bgcomp, a.bglocal, a.nb, a.bgoff, a.P,
                                          a.moff, a.M, a.BG);
  if (a.m > 0) {
    unsigned g = blocks_for(a.m);
    if (g > 8192) g = 8192;
    k_bg_edges<<<g, 256, 0, s>>>(a.m, a.eu, a.ev, a.w, a.comp, a.local, a.bgoff, a.Vp, a.BG);
  }
  LAUNCH_CHECK();
}

hipError_t launch_query(const QueryArgs& a, hipStream_t s) {
  if (a.q <= 0) return hipSuccess;
  const int64_t blocks = (a.q + 7) / 8;  // 8 pairs per workgroup
  k_query<<<(unsigned)blocks, 256, 0, s>>>(a.q, a.v1, a.v2, a.out, a.n, a.vrec, a.M, a.H,
                                           a.share_comps);
  LAUNCH_CHECK();
}

hipError_t launch_adjacency(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                            unsigned long long* deg, int64_t* rowptr, int2* adj, hipStream_t s) {
  // deg: n counters (zeroed by the caller), then reused as the fill cursors
  if (m > 0) {
    unsigned g = blocks_for(m);
    if (g > 8192) g = 8192;
    k_adj_count<<<g, 256, 0, s>>>(m, eu, ev, deg);
  }
  k_adj_scan<<<1, 256, 0, s>>>(n, deg, rowptr);
  hipError_t e = hipMemcpyAsync(deg, rowptr, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  if (m > 0) {
    unsigned g = blocks_for(m);
    if (g > 8192) g = 8192;
    k_adj_fill<<<g, 256, 0, s>>>(m, eu, ev, deg, adj);
  }
  LAUNCH_CHECK();
}

hipError_t launch_paths(const QueryArgs& a, int32_t max_len, const int64_t* rowptr, const int2* adj,
                        const int32_t* wts, int32_t* paths, int32_t* lens, hipStream_t s) {
  if (a.q <= 0) return hipSuccess;
  const int64_t blocks = (a.q + 7) / 8;  // 8 paths per workgroup
  k_paths<<<(unsigned)blocks, 256, 0, s>>>(a.q, a.v1, a.v2, max_len, a.n, a.vrec, a.M, a.H,
                                           a.share_comps, rowptr, adj, wts, paths, lens);
  LAUNCH_CHECK();
}

}  // namespace spq
