// Exactness certificate for graphs whose total edge weight reaches INF.
//
// Every stored distance is min(exact distance, INF) (see tiles.h), so the
// only possible error is a finite distance at or above INF shown as INF.  The
// build proves that none exists:
//   (i)   every component's edge weights sum below INF, so APSP(C) is exact;
//   (ii)  no BG entry is INF between two boundary vertices that are connected
//         in G (connected components computed here), so BG is exact;
//   (iii) 2 * max finite APSP(C) entry + max finite BG entry < INF, so every
//         sum a query forms on an optimal decomposition stays below INF.
// Under (i)-(iii) all answers are exact; otherwise the build reports
// SPQ_ERANGE.
#include "spq_internal.h"
#include "tiles.h"

namespace spq {

__global__ void k_cc_init(int32_t n, int32_t* __restrict__ label) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    label[v] = (int32_t)v;
}

// Labels only decrease and always point to a smaller or equal id, so every
// chain ends at a root.
__device__ __forceinline__ int32_t cc_root(const int32_t* label, int32_t x) {
  for (;;) {
    const int32_t p = __atomic_load_n(label + x, __ATOMIC_RELAXED);
    if (p == x) return x;
    x = p;
  }
}

// Hooks the larger root of every edge under the smaller one.
__global__ void k_cc_hook(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                          int32_t* label, u32* __restrict__ changed) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = cc_root(label, eu[e]), b = cc_root(label, ev[e]);
    if (a != b) {
      atomicMin(label + max(a, b), min(a, b));
      atomicOr(changed, 1u);
    }
  }
}

__global__ void k_cc_flatten(int32_t n, int32_t* label) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    label[v] = cc_root(label, (int32_t)v);
}

__global__ void k_bg_label(int32_t V, const int32_t* __restrict__ bgvert, const int32_t* __restrict__ label,
                           int32_t* __restrict__ bglabel) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < V;
       x += (int64_t)gridDim.x * blockDim.x)
    bglabel[x] = label[bgvert[x]];
}

__device__ __forceinline__ u32 wave_max(u32 v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, (u32)__shfl_xor((int)v, o));
  return v;
}

// Largest entry below INF of a contiguous array.
__global__ void k_max_finite(int64_t count, const u32* __restrict__ a, u32* __restrict__ out) {
  u32 best = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const u32 v = a[i];
    if (v < INF) best = max(best, v);
  }
  best = wave_max(best);
  if ((threadIdx.x & 63) == 0) atomicMax(out, best);
}

// Flat BG: rows p < V, columns q < V.
__global__ void k_check_flat(int32_t V, int64_t Vp, const u32* __restrict__ BG,
                             const int32_t* __restrict__ bglabel, u32* __restrict__ bad,
                             u32* __restrict__ mbg) {
  const int64_t p = blockIdx.x;
  const u32* row = BG + p * Vp;
  const int32_t lp = bglabel[p];
  u32 best = 0, wrong = 0;
  for (int64_t q = threadIdx.x; q < V; q += blockDim.x) {
    const u32 v = row[q];
    if (v < INF) best = max(best, v);
    else if (bglabel[q] == lp) wrong = 1;
  }
  best = wave_max(best);
  wrong = wave_max(wrong);
  if ((threadIdx.x & 63) == 0) {
    if (best) atomicMax(mbg, best);
    if (wrong) atomicOr(bad, 1u);
  }
}

// Two-level store: block (pair (s1, s2), 16-row chunk of group s1), s1 <= s2.
__global__ void k_check_hier(int32_t ngroups, const int32_t* __restrict__ gV,
                             const int32_t* __restrict__ gbg0, const int64_t* __restrict__ pairbase,
                             const int32_t* __restrict__ bgrow, const int32_t* __restrict__ bgnb,
                             const int32_t* __restrict__ bglocal, const int32_t* __restrict__ bglabel,
                             const u32* __restrict__ H, u32* __restrict__ bad, u32* __restrict__ mbg) {
  const int32_t s1 = (int32_t)(blockIdx.x / ngroups), s2 = (int32_t)(blockIdx.x % ngroups);
  if (s1 > s2) return;
  const int32_t V1 = gV[s1], V2 = gV[s2], g1 = gbg0[s1], g2 = gbg0[s2];
  const u32* base = H + pairbase[(int64_t)s1 * ngroups + s2];
  u32 best = 0, wrong = 0;
  for (int32_t r = 0; r < 16; r++) {
    const int32_t x = (int32_t)blockIdx.y * 16 + r;
    if (x >= V1) break;
    const int32_t xg = g1 + x;
    const int64_t rb = (int64_t)bgrow[xg] * V2;
    const int64_t nbx = bgnb[xg], locx = bglocal[xg];
    const int32_t lx = bglabel[xg];
    for (int32_t y = threadIdx.x; y < V2; y += blockDim.x) {
      const int32_t yg = g2 + y;
      const u32 v = base[rb + nbx * bgrow[yg] + locx * bgnb[yg] + bglocal[yg]];
      if (v < INF) best = max(best, v);
      else if (bglabel[yg] == lx) wrong = 1;
    }
  }
  best = wave_max(best);
  wrong = wave_max(wrong);
  if ((threadIdx.x & 63) == 0) {
    if (best) atomicMax(mbg, best);
    if (wrong) atomicOr(bad, 1u);
  }
}

static inline unsigned rblocks(int64_t items) {
  int64_t b = (items + 255) / 256;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (unsigned)b;
}

hipError_t launch_cc_init(int32_t n, int32_t* label, hipStream_t s) {
  k_cc_init<<<rblocks(n), 256, 0, s>>>(n, label);
  return hipGetLastError();
}

hipError_t launch_cc_round(int64_t m, const int32_t* eu, const int32_t* ev, int32_t n, int32_t* label,
                           u32* changed, hipStream_t s) {
  if (m > 0) k_cc_hook<<<rblocks(m), 256, 0, s>>>(m, eu, ev, label, changed);
  k_cc_flatten<<<rblocks(n), 256, 0, s>>>(n, label);
  return hipGetLastError();
}

hipError_t launch_bg_label(int32_t V, const int32_t* bgvert, const int32_t* label, int32_t* bglabel,
                           hipStream_t s) {
  if (V > 0) k_bg_label<<<rblocks(V), 256, 0, s>>>(V, bgvert, label, bglabel);
  return hipGetLastError();
}

hipError_t launch_certificate(const CertArgs& a, hipStream_t s) {
  if (a.comp_elems > 0) k_max_finite<<<rblocks(a.comp_elems), 256, 0, s>>>(a.comp_elems, a.M, a.mc);
  if (a.V > 0 && !a.bg_checked) {
    if (a.H) {
      dim3 grid((unsigned)((int64_t)a.ngroups * a.ngroups), (unsigned)((a.Vgp + 15) / 16));
      k_check_hier<<<grid, 256, 0, s>>>(a.ngroups, a.gV, a.gbg0, a.pairbase, a.bgrow, a.bgnb,
                                         a.bglocal, a.bglabel, a.H, a.bad, a.mbg);
    } else {
      k_check_flat<<<(unsigned)a.V, 256, 0, s>>>(a.V, a.Vp, a.BG, a.bglabel, a.bad, a.mbg);
    }
  }
  return hipGetLastError();
}

}  // namespace spq
