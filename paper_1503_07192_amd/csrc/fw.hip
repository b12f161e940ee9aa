// Blocked Floyd-Warshall (min-plus) on dense symmetric matrices: the
// closure of BG (Algorithm 1, Phase 3, by Floyd-Warshall instead of the
// paper's Dijkstra), of large components (Phase 2) and of the group and
// level-2/3 matrices of the two-level method.
#include "spq_internal.h"
#include "tiles.h"

namespace spq {

#define LAUNCH_CHECK() return hipGetLastError()

// Blocked Floyd-Warshall on one symmetric matrix, round r of nt:
//   k_fw_diag   closes the diagonal tile (r, r)
//   k_fw_panel  tile (r, j) = D (x) tile (r, j) for j != r, stored twice
//               (as (r, j) and transposed as (j, r))
//   k_fw_inner  tile (i, j) = min(tile (i, j), tile (r, i)^T (x) tile (r, j))
//
// A batch of equally sized matrices is handled by blockIdx.y: matrix y starts
// gstride elements after matrix y-1.
template <int T>
__global__ __launch_bounds__(256) void k_fw_diag(u32* __restrict__ A, int64_t ld, int r,
                                                 int64_t gstride) {
  __shared__ __attribute__((aligned(16))) u32 rb[4 * T];
  A += (int64_t)blockIdx.y * gstride;
  u32 t[T / 16][T / 16];
  u32* D = A + (int64_t)r * T * ld + (int64_t)r * T;
  tile_load<T>(t, D, ld);
  fw_tile<T>(t, rb);
  tile_store<T>(t, D, ld);
}

template <int T>
__global__ __launch_bounds__(256) void k_fw_panel(u32* __restrict__ A, int64_t ld, int r,
                                                  int64_t gstride) {
  __shared__ __attribute__((aligned(16))) u32 sD[T * T];
  __shared__ __attribute__((aligned(16))) u32 sB[T * T];
  A += (int64_t)blockIdx.y * gstride;
  const int j = (int)blockIdx.x + ((int)blockIdx.x >= r);
  u32 t[T / 16][T / 16];
  tile_load<T>(t, A + (int64_t)r * T * ld + (int64_t)r * T, ld);
  tile_to_lds<T>(t, sD);
  u32* Rj = A + (int64_t)r * T * ld + (int64_t)j * T;
  tile_load<T>(t, Rj, ld);
  tile_to_lds<T>(t, sB);
  __syncthreads();
  minplus_lds<T>(t, sD, sB, T);
  tile_store<T>(t, Rj, ld);
  tile_store_t<T>(t, A + (int64_t)j * T * ld + (int64_t)r * T, ld);
}

// Upper-triangle enumeration: block b -> (bi, bj), 0 <= bi <= bj < m, row by
// row (row bi holds m - bi blocks).
__device__ __forceinline__ void tri_index(int b, int m, int& bi, int& bj) {
  const float fm = 2.0f * m + 1.0f;
  int i = (int)((fm - sqrtf(fm * fm - 8.0f * (float)b)) * 0.5f);
  if (i < 0) i = 0;
  if (i > m - 1) i = m - 1;
  while (i > 0 && i * (2 * m - i + 1) / 2 > b) i--;
  while (i + 1 < m && (i + 1) * (2 * m - i) / 2 <= b) i++;
  bi = i;
  bj = i + (b - i * (2 * m - i + 1) / 2);
}

// Interior tiles.  The matrix is symmetric, so only tiles (i, j) with i <= j
// are computed; tile (j, i) receives the transpose.  The k dimension is
// streamed through LDS in chunks of KC rows of the two operand tiles (double
// buffered, next chunk prefetched into registers while the current one is
// consumed).
#ifdef SPQ_INNER_WPE
#define SPQ_INNER_ATTR __attribute__((amdgpu_waves_per_eu(SPQ_INNER_WPE, SPQ_INNER_WPE)))
#else
#define SPQ_INNER_ATTR
#endif
//
// part selects the tiles of the launch:
//   0  every interior tile (i <= j, both != r)
//   1  the tiles of row/column r+1 only: (i, r+1) for i <= r+1, i != r, and
//      (r+1, j) for j > r+1 (what the next round's pivot row needs)
//   2  every interior tile not in part 1
template <int T, int KC>
__global__ __launch_bounds__(256) SPQ_INNER_ATTR void k_fw_inner(u32* __restrict__ A, int64_t ld, int r, int nt,
                                                                int64_t gstride, int part) {
  constexpr int Q = KC * T / 4 / 256;  // uint4 per thread per operand chunk
  static_assert(Q >= 1 && KC * T / 4 % 256 == 0, "chunk must split evenly");
  __shared__ __attribute__((aligned(16))) u32 sA[2][KC * T];
  __shared__ __attribute__((aligned(16))) u32 sB[2][KC * T];
  A += (int64_t)blockIdx.y * gstride;
  int i, j;
  const int b = (int)blockIdx.x;
  if (part == 0) {
    int bi, bj;
    tri_index(b, nt - 1, bi, bj);
    i = bi + (bi >= r);
    j = bj + (bj >= r);
  } else if (part == 1) {
    const int p = r + 1;  // nt - 1 tiles
    if (b <= r) {         // (i, p) for i in [0, p], i != r; b == r gives (p, p)
      i = b + (b >= r ? 1 : 0);
      j = p;
    } else {              // (p, j) for j in (p, nt)
      i = p;
      j = b + 1;
    }
  } else {
    int bi, bj;           // triangle over indices other than r and r+1
    tri_index(b, nt - 2, bi, bj);
    i = bi + (bi >= r ? 2 : 0);
    j = bj + (bj >= r ? 2 : 0);
  }
  const u32* Ar = A + (int64_t)r * T * ld + (int64_t)i * T;  // tile (r, i)
  const u32* Br = A + (int64_t)r * T * ld + (int64_t)j * T;  // tile (r, j)
  u32* Cij = A + (int64_t)i * T * ld + (int64_t)j * T;
  u32 t[T / 16][T / 16];
  tile_load<T>(t, Cij, ld);
  uint4 pa[Q], pb[Q];
  // chunk 0 straight to LDS buffer 0
#pragma unroll
  for (int s = 0; s < Q; s++) {
    const int e = threadIdx.x + s * 256;
    const int row = e / (T / 4), c4 = e % (T / 4);
    pa[s] = *reinterpret_cast<const uint4*>(Ar + (int64_t)row * ld + c4 * 4);
    pb[s] = *reinterpret_cast<const uint4*>(Br + (int64_t)row * ld + c4 * 4);
  }
#pragma unroll
  for (int s = 0; s < Q; s++) {
    const int e = threadIdx.x + s * 256;
    reinterpret_cast<uint4*>(sA[0])[e] = pa[s];
    reinterpret_cast<uint4*>(sB[0])[e] = pb[s];
  }
  __syncthreads();
  // The chunk loop stays rolled: unrolled, it needed 136 VGPRs (three waves
  // per SIMD); rolled it fits 128 (four waves, 3.5% faster on a 27,904-wide
  // matrix).  The last chunk reloads itself into the idle buffer (unused), so
  // the prefetch needs no branch.
  constexpr int NCH = T / KC;
#pragma unroll 1
  for (int ch = 0; ch < NCH; ch++) {
    const int kc = (ch + 1 < NCH ? ch + 1 : ch) * KC;
#pragma unroll
    for (int s = 0; s < Q; s++) {
      const int e = threadIdx.x + s * 256;
      const int row = e / (T / 4), c4 = e % (T / 4);
      pa[s] = *reinterpret_cast<const uint4*>(Ar + (int64_t)(kc + row) * ld + c4 * 4);
      pb[s] = *reinterpret_cast<const uint4*>(Br + (int64_t)(kc + row) * ld + c4 * 4);
    }
    minplus_lds<T>(t, sA[ch & 1], sB[ch & 1], KC);
#pragma unroll
    for (int s = 0; s < Q; s++) {
      const int e = threadIdx.x + s * 256;
      reinterpret_cast<uint4*>(sA[(ch + 1) & 1])[e] = pa[s];
      reinterpret_cast<uint4*>(sB[(ch + 1) & 1])[e] = pb[s];
    }
    __syncthreads();
  }
  tile_store<T>(t, Cij, ld);
  if (i != j) tile_store_t<T>(t, A + (int64_t)j * T * ld + (int64_t)i * T, ld);
}

#ifndef SPQ_INNER_KC
#define SPQ_INNER_KC 16
#endif

template <int T, int KC>
static hipError_t fw_rounds(u32* A, int64_t ld, int nt, int batch, int64_t gstride, hipStream_t s,
                           hipEvent_t* ev) {
  for (int r = 0; r < nt; r++) {
    k_fw_diag<T><<<dim3(1, batch), 256, 0, s>>>(A, ld, r, gstride);
    if (nt > 1) {
      k_fw_panel<T><<<dim3(nt - 1, batch), 256, 0, s>>>(A, ld, r, gstride);
      if (ev) {
        hipError_t e = hipEventRecord(ev[2 * r], s);
        if (e != hipSuccess) return e;
      }
      k_fw_inner<T, KC><<<dim3((unsigned)((nt - 1) * nt / 2), batch), 256, 0, s>>>(
          A, ld, r, nt, gstride, 0);
      if (ev) {
        hipError_t e = hipEventRecord(ev[2 * r + 1], s);
        if (e != hipSuccess) return e;
      }
    }
  }
  LAUNCH_CHECK();
}

// The same rounds with a lookahead: the interior tiles of row/column r+1 go
// first (part 1); as soon as they are done, round r+1's diagonal and panel
// run on the side stream while the rest of round r's interior (part 2) runs
// on the main stream.  Part 2 neither reads nor writes a tile that round
// r+1's diagonal or panel touches (row/column r+1 and the tiles (r, r+1),
// (r+1, r)), so the two overlap safely.  ev (optional) gets one pair per
// round around parts 1 + 2.
template <int T, int KC>
static hipError_t fw_rounds_lookahead(u32* A, int64_t ld, int nt, hipStream_t s, hipStream_t side,
                                      hipEvent_t* sync, hipEvent_t* ev) {
#define CHK(x)                              \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)
  // sync[0] = side stream may start round r+1 (part 1 of round r done);
  // sync[1] = main stream may start round r+1's interior (its panel done)
  CHK(hipEventRecord(sync[0], s));
  CHK(hipStreamWaitEvent(side, sync[0], 0));
  k_fw_diag<T><<<1, 256, 0, side>>>(A, ld, 0, 0);
  k_fw_panel<T><<<nt - 1, 256, 0, side>>>(A, ld, 0, 0);
  CHK(hipEventRecord(sync[1], side));
  for (int r = 0; r < nt; r++) {
    CHK(hipStreamWaitEvent(s, sync[1], 0));
    if (ev) CHK(hipEventRecord(ev[2 * r], s));
    if (r + 1 < nt) {
      k_fw_inner<T, KC><<<(unsigned)nt - 1, 256, 0, s>>>(A, ld, r, nt, 0, 1);
      CHK(hipEventRecord(sync[0], s));
      CHK(hipStreamWaitEvent(side, sync[0], 0));
      k_fw_diag<T><<<1, 256, 0, side>>>(A, ld, r + 1, 0);
      k_fw_panel<T><<<nt - 1, 256, 0, side>>>(A, ld, r + 1, 0);
      if (nt > 2)
        k_fw_inner<T, KC><<<(unsigned)((nt - 2) * (nt - 1) / 2), 256, 0, s>>>(A, ld, r, nt, 0, 2);
      CHK(hipEventRecord(sync[1], side));
    } else {
      // last round: nothing to look ahead to
      k_fw_inner<T, KC><<<(unsigned)((nt - 1) * nt / 2), 256, 0, s>>>(A, ld, r, nt, 0, 0);
    }
    if (ev) CHK(hipEventRecord(ev[2 * r + 1], s));
  }
#undef CHK
  LAUNCH_CHECK();
}

hipError_t launch_dense_fw(u32* A, int64_t ld, int tile, int nt, hipStream_t s, hipEvent_t* ev,
                           int kc) {
  return launch_dense_fw_batch(A, ld, tile, nt, 1, 0, s, ev, kc);
}

hipError_t launch_dense_fw_lookahead(u32* A, int64_t ld, int tile, int nt, hipStream_t s,
                                     hipStream_t side, hipEvent_t* sync, hipEvent_t* ev, int kc) {
  if (nt <= 1) return launch_dense_fw(A, ld, tile, nt, s, ev, kc);
  if (kc == 0) kc = SPQ_INNER_KC;
  if (tile == 64)
    return kc == 32 ? fw_rounds_lookahead<64, 32>(A, ld, nt, s, side, sync, ev)
                    : fw_rounds_lookahead<64, 16>(A, ld, nt, s, side, sync, ev);
  return kc == 32 ? fw_rounds_lookahead<128, 32>(A, ld, nt, s, side, sync, ev)
                  : fw_rounds_lookahead<128, 16>(A, ld, nt, s, side, sync, ev);
}

// kc: K chunk of the interior-tile kernel (16 or 32; 0 = SPQ_INNER_KC)
hipError_t launch_dense_fw_batch(u32* A, int64_t ld, int tile, int nt, int batch, int64_t gstride,
                                 hipStream_t s, hipEvent_t* ev, int kc) {
  if (nt <= 0 || batch <= 0) return hipSuccess;
  if (kc == 0) kc = SPQ_INNER_KC;
  if (tile == 64)
    return kc == 32 ? fw_rounds<64, 32>(A, ld, nt, batch, gstride, s, ev)
                    : fw_rounds<64, 16>(A, ld, nt, batch, gstride, s, ev);
  return kc == 32 ? fw_rounds<128, 32>(A, ld, nt, batch, gstride, s, ev)
                  : fw_rounds<128, 16>(A, ld, nt, batch, gstride, s, ev);
}

double dense_fw_exec_relax(int64_t nt, int tile) {
  const double t3 = (double)tile * tile * tile;
  return (double)nt * t3 * (1.0 + (nt - 1) + (double)(nt - 1) * nt / 2.0);
}

}  // namespace spq
