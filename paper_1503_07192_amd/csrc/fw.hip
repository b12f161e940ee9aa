// Blocked Floyd-Warshall (min-plus) on dense symmetric matrices: the
// closure of BG (Algorithm 1, Phase 3, by Floyd-Warshall instead of the
// paper's Dijkstra), of large components (Phase 2) and of the group and
// level-2/3 matrices of the two-level method.
#include "spq_internal.h"
#include "tiles.h"

#include <vector>

namespace spq {

#define LAUNCH_CHECK() return hipGetLastError()

// Blocked Floyd-Warshall on one symmetric matrix of nt x nt tiles, in rounds
// over pivot blocks of one, two or four tiles (the tiles left at the end form
// smaller blocks):
//   close    the pivot block: k_fw_diag for one tile; a larger block by the
//            same rounds on the sub-matrix, over blocks of half its size
//   panel    tile (a, j), a in the block, j outside it: tile (a, j) =
//            D (x) tile (a, j), stored twice (as (a, j) and transposed as
//            (j, a)); k_fw_inner part 3 (k_fw_panel in fw_rounds, the
//            one-tile rounds of a batch)
//   interior tile (i, j) = min(tile (i, j),
//            (block rows, tile i)^T (x) (block rows, tile j)), k_fw_inner
// A two-tile block doubles the K of every interior product (256 instead of
// 128 for 128-tiles): the fixed cost of a tile (loading and storing C) is
// spread over twice the relaxations, and there are half as many rounds.
//
// A batch of equally sized matrices (one-tile blocks only) is handled by
// blockIdx.y: matrix y starts gstride elements after matrix y-1.
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
// are computed; tile (j, i) receives the transpose.  The k dimension (the
// PT * T rows of the pivot block) is streamed through LDS in chunks of KC rows
// of the two operand tiles (double buffered, next chunk prefetched into
// registers while the current one is consumed).
#ifdef SPQ_INNER_WPE
#define SPQ_INNER_ATTR __attribute__((amdgpu_waves_per_eu(SPQ_INNER_WPE, SPQ_INNER_WPE)))
#else
#define SPQ_INNER_ATTR
#endif
//
// The pivot block is tiles [c0, c0 + PT); nn = tiles of the next block
// (parts 1 and 2).  part selects the tiles of the launch:
//   0  every tile outside the pivot block (i <= j)
//   1  the tiles with a row or column in the next block (what the next
//      round's diagonal and panel read)
//   2  every tile outside both blocks
//   3  the panel: (a, j) for a in the pivot block, j outside it (PT = 2)
template <int PT>
__device__ __forceinline__ void inner_tile(int part, int b, int c0, int nt, int nn, int& i, int& j) {
  int bi, bj;
  if (part == 0) {
    tri_index(b, nt - PT, bi, bj);
    i = bi + (bi >= c0 ? PT : 0);
    j = bj + (bj >= c0 ? PT : 0);
  } else if (part == 1) {
    const int no = nt - PT - nn;  // tiles outside both blocks
    if (b < nn * no) {
      const int x = c0 + PT + b / no, o = b % no;
      const int y = o + (o >= c0 ? PT + nn : 0);
      i = min(x, y);
      j = max(x, y);
    } else {
      tri_index(b - nn * no, nn, bi, bj);
      i = c0 + PT + bi;
      j = c0 + PT + bj;
    }
  } else if (part == 2) {
    tri_index(b, nt - PT - nn, bi, bj);
    i = bi + (bi >= c0 ? PT + nn : 0);
    j = bj + (bj >= c0 ? PT + nn : 0);
  } else {
    const int m = nt - PT, o = b % m;
    i = c0 + b / m;
    j = o + (o >= c0 ? PT : 0);
  }
}

template <int T, int KC, int PT>
__global__ __launch_bounds__(256) SPQ_INNER_ATTR void k_fw_inner(u32* __restrict__ A, int64_t ld, int c0, int nt,
                                                                int64_t gstride, int part, int nn) {
  constexpr int Q = KC * T / 4 / 256;  // uint4 per thread per operand chunk
  static_assert(Q >= 1 && KC * T / 4 % 256 == 0, "chunk must split evenly");
  __shared__ __attribute__((aligned(16))) u32 sA[2][KC * T];
  __shared__ __attribute__((aligned(16))) u32 sB[2][KC * T];
  A += (int64_t)blockIdx.y * gstride;
  int i, j;
  inner_tile<PT>(part, (int)blockIdx.x, c0, nt, nn, i, j);
  const u32* Ar = A + (int64_t)c0 * T * ld + (int64_t)i * T;  // block rows, tile column i
  const u32* Br = A + (int64_t)c0 * T * ld + (int64_t)j * T;  // block rows, tile column j
  u32* Cij = A + (int64_t)i * T * ld + (int64_t)j * T;
  u32 t[T / 16][T / 16];
  tile_load<T>(t, Cij, ld);
  // The operand chunks go from global memory straight to LDS
  // (global_load_lds_dwordx4, gfx950): no staging registers and no LDS
  // stores.  Element e (in 16-byte units) of a chunk is row e / (T/4),
  // column 4 (e % (T/4)); lane l of wave w loads e = s*256 + w*64 + l, and a
  // wave's 64 lanes fill 1 KB of LDS in that order.  A chunk is complete once
  // every wave's loads have arrived: vmcnt(0), then the barrier.
  const int wv = (int)threadIdx.x >> 6;
  auto load_chunk = [&](int kc, int buf) {
#pragma unroll
    for (int s = 0; s < Q; s++) {
      const int e = threadIdx.x + s * 256;
      const int row = e / (T / 4), c4 = e % (T / 4);
      const int64_t off = (int64_t)(kc + row) * ld + c4 * 4;
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(Ar + off),
                                       (__attribute__((address_space(3))) void*)(&sA[buf][(s * 256 + wv * 64) * 4]),
                                       16, 0, 0);
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(Br + off),
                                       (__attribute__((address_space(3))) void*)(&sB[buf][(s * 256 + wv * 64) * 4]),
                                       16, 0, 0);
    }
  };
  load_chunk(0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // The chunk loop stays rolled (unrolled, the staged version needed 136
  // VGPRs and three waves per SIMD).
  constexpr int NCH = PT * T / KC;
#pragma unroll 1
  for (int ch = 0; ch < NCH; ch++) {
    if (ch + 1 < NCH) load_chunk((ch + 1) * KC, (ch + 1) & 1);
    minplus_lds<T>(t, sA[ch & 1], sB[ch & 1], KC);
    __builtin_amdgcn_s_waitcnt(0);
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
      k_fw_inner<T, KC, 1><<<dim3((unsigned)((nt - 1) * nt / 2), batch), 256, 0, s>>>(
          A, ld, r, nt, gstride, 0, 1);
      if (ev) {
        hipError_t e = hipEventRecord(ev[2 * r + 1], s);
        if (e != hipSuccess) return e;
      }
    }
  }
  LAUNCH_CHECK();
}

// Pivot blocks of a single matrix: pivot_tiles (1, 2 or 4) tiles each; the
// tiles left at the end form blocks of two and one.
struct FwBlock {
  int c0, pt;
};

static int fw_blocks(int nt, int pivot_tiles, FwBlock* out) {
  int nb = 0;
  for (int c0 = 0; c0 < nt; nb++) {
    int pt = pivot_tiles;
    while (pt > nt - c0) pt >>= 1;
    if (out) out[nb] = FwBlock{c0, pt};
    c0 += pt;
  }
  return nb;
}

static int64_t tri_count(int64_t m) { return m > 0 ? m * (m + 1) / 2 : 0; }

// tiles of an interior launch of block b (parts 0-2; nn = next block's tiles)
static int64_t inner_count(int nt, FwBlock b, int part, int nn) {
  if (part == 0) return tri_count(nt - b.pt);
  if (part == 1) return (int64_t)nn * (nt - b.pt - nn) + tri_count(nn);
  return tri_count(nt - b.pt - nn);
}

// `batch` equally sized matrices, gstride elements apart (blockIdx.y)
struct FwBatch {
  int batch;
  int64_t gstride;
};

template <int T, int KC>
static hipError_t fw_rounds_blocks(u32* A, int64_t ld, int nt, int pivot_tiles, FwBatch bt,
                                   hipStream_t s, hipEvent_t* ev);

// Closes the diagonal block: one tile in one workgroup (k_fw_diag); a block
// of two or four tiles by the rounds of this file on the sub-matrix, over
// blocks of half its size.  Every launch of a block closure is small (one to
// six workgroups of 32 KB LDS at most), so beside a running interior launch
// it finds room on a CU at once; one workgroup holding two tiles in LDS
// (130 KB) waited for a whole CU to drain, about as long as the interior.
template <int T, int KC>
static hipError_t fw_close(u32* A, int64_t ld, FwBlock b, FwBatch bt, hipStream_t s) {
  if (b.pt == 1) {
    k_fw_diag<T><<<dim3(1, bt.batch), 256, 0, s>>>(A, ld, b.c0, bt.gstride);
    return hipGetLastError();
  }
  return fw_rounds_blocks<T, KC>(A + (int64_t)b.c0 * T * ld + (int64_t)b.c0 * T, ld, b.pt, b.pt / 2,
                                 bt, s, nullptr);
}

// The panel of block b: tiles (a, j), a in the block, j outside it, by the
// interior kernel (part 3; 32 KB LDS, not k_fw_panel's 128 KB, for the same
// reason as above).
template <int T, int KC>
static hipError_t fw_panel(u32* A, int64_t ld, int nt, FwBlock b, FwBatch bt, hipStream_t s) {
  if (nt <= b.pt) return hipSuccess;
  const dim3 grid((unsigned)(b.pt * (nt - b.pt)), (unsigned)bt.batch);
  if (b.pt == 1)
    k_fw_inner<T, KC, 1><<<grid, 256, 0, s>>>(A, ld, b.c0, nt, bt.gstride, 3, 0);
  else if (b.pt == 2)
    k_fw_inner<T, KC, 2><<<grid, 256, 0, s>>>(A, ld, b.c0, nt, bt.gstride, 3, 0);
  else
    k_fw_inner<T, KC, 4><<<grid, 256, 0, s>>>(A, ld, b.c0, nt, bt.gstride, 3, 0);
  return hipGetLastError();
}

template <int T, int KC>
static hipError_t fw_inner(u32* A, int64_t ld, int nt, FwBlock b, int part, int nn, FwBatch bt,
                           hipStream_t s) {
  const int64_t count = inner_count(nt, b, part, nn);
  if (count <= 0) return hipSuccess;
  const dim3 grid((unsigned)count, (unsigned)bt.batch);
  if (b.pt == 1)
    k_fw_inner<T, KC, 1><<<grid, 256, 0, s>>>(A, ld, b.c0, nt, bt.gstride, part, nn);
  else if (b.pt == 2)
    k_fw_inner<T, KC, 2><<<grid, 256, 0, s>>>(A, ld, b.c0, nt, bt.gstride, part, nn);
  else
    k_fw_inner<T, KC, 4><<<grid, 256, 0, s>>>(A, ld, b.c0, nt, bt.gstride, part, nn);
  return hipGetLastError();
}

#define CHK(x)                              \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

// Rounds over the pivot blocks on one stream (a batch of matrices at once).
// ev (optional) gets one pair per round around its interior launch.
template <int T, int KC>
static hipError_t fw_rounds_blocks(u32* A, int64_t ld, int nt, int pivot_tiles, FwBatch bt,
                                   hipStream_t s, hipEvent_t* ev) {
  std::vector<FwBlock> blk(fw_blocks(nt, pivot_tiles, nullptr));
  fw_blocks(nt, pivot_tiles, blk.data());
  for (size_t q = 0; q < blk.size(); q++) {
    CHK((fw_close<T, KC>(A, ld, blk[q], bt, s)));
    if (nt <= blk[q].pt) continue;
    CHK((fw_panel<T, KC>(A, ld, nt, blk[q], bt, s)));
    if (ev) CHK(hipEventRecord(ev[2 * q], s));
    CHK((fw_inner<T, KC>(A, ld, nt, blk[q], 0, 0, bt, s)));
    if (ev) CHK(hipEventRecord(ev[2 * q + 1], s));
  }
  return hipSuccess;
}

// The same rounds with a lookahead: the interior tiles with a row or column
// in the next pivot block go first (part 1); as soon as they are done, the
// next round's diagonal block and panel run on the side stream while the rest
// of this round's interior (part 2) runs on the main stream.  Part 2 neither
// reads nor writes a tile that the next round's diagonal or panel touches
// (rows and columns of the next block: the panel also writes the tiles of the
// current block's rows in those columns, which part 2 does not read), so the
// two overlap safely.  A batch of matrices runs the same rounds side by side
// (the argument holds for each).  With a third stream p1, part 1 runs there
// beside part 2 instead of before it (part 1 alone leaves workgroup slots
// idle); the round still ends only when both are done.  ev (optional) gets
// one pair per round around parts 1 + 2.
template <int T, int KC>
static hipError_t fw_rounds_lookahead(u32* A, int64_t ld, int nt, int pivot_tiles, FwBatch bt,
                                      hipStream_t s, hipStream_t side, hipStream_t p1,
                                      hipEvent_t* sync, hipEvent_t* ev) {
  std::vector<FwBlock> blk(fw_blocks(nt, pivot_tiles, nullptr));
  fw_blocks(nt, pivot_tiles, blk.data());
  // sync[0] = side stream may start the next round (part 1 of this one done);
  // sync[1] = main stream may start the next round's interior (its panel done);
  // sync[2] (with p1) = p1 may start this round's part 1
  CHK(hipEventRecord(sync[0], s));
  CHK(hipStreamWaitEvent(side, sync[0], 0));
  CHK((fw_close<T, KC>(A, ld, blk[0], bt, side)));
  CHK((fw_panel<T, KC>(A, ld, nt, blk[0], bt, side)));
  CHK(hipEventRecord(sync[1], side));
  for (size_t q = 0; q < blk.size(); q++) {
    CHK(hipStreamWaitEvent(s, sync[1], 0));
    if (nt <= blk[q].pt) continue;  // a single block: closed, nothing else
    if (ev) CHK(hipEventRecord(ev[2 * q], s));
    if (q + 1 < blk.size()) {
      const int nn = blk[q + 1].pt;
      hipStream_t s1 = s;
      if (p1) {
        CHK(hipEventRecord(sync[2], s));
        CHK(hipStreamWaitEvent(p1, sync[2], 0));
        s1 = p1;
      }
      CHK((fw_inner<T, KC>(A, ld, nt, blk[q], 1, nn, bt, s1)));
      CHK(hipEventRecord(sync[0], s1));
      CHK(hipStreamWaitEvent(side, sync[0], 0));
      CHK((fw_close<T, KC>(A, ld, blk[q + 1], bt, side)));
      CHK((fw_panel<T, KC>(A, ld, nt, blk[q + 1], bt, side)));
      CHK((fw_inner<T, KC>(A, ld, nt, blk[q], 2, nn, bt, s)));
      CHK(hipEventRecord(sync[1], side));
      if (p1) CHK(hipStreamWaitEvent(s, sync[0], 0));  // the round ends with part 1 too
    } else {
      // last round: nothing to look ahead to
      CHK((fw_inner<T, KC>(A, ld, nt, blk[q], 0, 0, bt, s)));
    }
    if (ev) CHK(hipEventRecord(ev[2 * q + 1], s));
  }
  return hipSuccess;
}

static int pivot_tiles_of(int tile, int pivot) { return pivot <= tile ? 1 : pivot / tile; }

int fw_rounds_count(int nt, int tile, int pivot) {
  return fw_blocks(nt, pivot_tiles_of(tile, pivot), nullptr);
}

hipError_t launch_dense_fw(u32* A, int64_t ld, int tile, int nt, hipStream_t s, hipEvent_t* ev,
                           int kc, int pivot) {
  return launch_dense_fw_batch(A, ld, tile, nt, 1, 0, s, ev, kc, pivot);
}

static hipError_t dense_lookahead(u32* A, int64_t ld, int tile, int nt, FwBatch bt, hipStream_t s,
                                  hipStream_t side, hipStream_t p1, hipEvent_t* sync,
                                  hipEvent_t* ev, int kc, int pivot) {
  if (nt <= 0 || bt.batch <= 0) return hipSuccess;
  const int pt = pivot_tiles_of(tile, pivot);
  if (kc == 0) kc = SPQ_INNER_KC;
  if (tile == 64)
    return kc == 32 ? fw_rounds_lookahead<64, 32>(A, ld, nt, pt, bt, s, side, p1, sync, ev)
                    : fw_rounds_lookahead<64, 16>(A, ld, nt, pt, bt, s, side, p1, sync, ev);
  return kc == 32 ? fw_rounds_lookahead<128, 32>(A, ld, nt, pt, bt, s, side, p1, sync, ev)
                  : fw_rounds_lookahead<128, 16>(A, ld, nt, pt, bt, s, side, p1, sync, ev);
}

hipError_t launch_dense_fw_lookahead(u32* A, int64_t ld, int tile, int nt, hipStream_t s,
                                     hipStream_t side, hipEvent_t* sync, hipEvent_t* ev, int kc,
                                     int pivot, hipStream_t p1) {
  return dense_lookahead(A, ld, tile, nt, FwBatch{1, 0}, s, side, p1, sync, ev, kc, pivot);
}

hipError_t launch_dense_fw_batch_lookahead(u32* A, int64_t ld, int tile, int nt, int batch,
                                           int64_t gstride, hipStream_t s, hipStream_t side,
                                           hipEvent_t* sync, hipEvent_t* ev, int kc, int pivot) {
  return dense_lookahead(A, ld, tile, nt, FwBatch{batch, gstride}, s, side, nullptr, sync, ev, kc,
                         pivot);
}
#undef CHK

// kc: K chunk of the interior-tile kernel (16 or 32; 0 = SPQ_INNER_KC)
hipError_t launch_dense_fw_batch(u32* A, int64_t ld, int tile, int nt, int batch, int64_t gstride,
                                 hipStream_t s, hipEvent_t* ev, int kc, int pivot) {
  if (nt <= 0 || batch <= 0) return hipSuccess;
  if (kc == 0) kc = SPQ_INNER_KC;
  const int pt = pivot_tiles_of(tile, pivot);
  if (pt > 1) {
    const FwBatch bt{batch, gstride};
    if (tile == 64)
      return kc == 32 ? fw_rounds_blocks<64, 32>(A, ld, nt, pt, bt, s, ev)
                      : fw_rounds_blocks<64, 16>(A, ld, nt, pt, bt, s, ev);
    return kc == 32 ? fw_rounds_blocks<128, 32>(A, ld, nt, pt, bt, s, ev)
                    : fw_rounds_blocks<128, 16>(A, ld, nt, pt, bt, s, ev);
  }
  if (tile == 64)
    return kc == 32 ? fw_rounds<64, 32>(A, ld, nt, batch, gstride, s, ev)
                    : fw_rounds<64, 16>(A, ld, nt, batch, gstride, s, ev);
  return kc == 32 ? fw_rounds<128, 32>(A, ld, nt, batch, gstride, s, ev)
                  : fw_rounds<128, 16>(A, ld, nt, batch, gstride, s, ev);
}

// Executed relaxations: per round the diagonal block (one tile: T^3; more:
// the rounds over half-size blocks on it), the panel (each of its tiles K =
// block rows) and the upper-triangle interior tiles; `inner` gets the
// interior part.
double dense_fw_exec_relax(int64_t nt, int tile, int pivot, double* inner) {
  const double t3 = (double)tile * tile * tile;
  const int ptiles = pivot_tiles_of(tile, pivot);
  std::vector<FwBlock> blk(fw_blocks((int)nt, ptiles, nullptr));
  fw_blocks((int)nt, ptiles, blk.data());
  double all = 0, in = 0;
  for (const FwBlock& b : blk) {
    all += b.pt == 1 ? t3 : dense_fw_exec_relax(b.pt, tile, b.pt / 2 * tile, nullptr);
    if (nt <= b.pt) continue;
    all += (double)b.pt * (nt - b.pt) * b.pt * t3;
    const double x = (double)tri_count(nt - b.pt) * b.pt * t3;
    all += x;
    in += x;
  }
  if (inner) *inner = in;
  return all;
}

}  // namespace spq
