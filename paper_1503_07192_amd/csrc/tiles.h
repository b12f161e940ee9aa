// Tile routines of the blocked Floyd-Warshall / min-plus kernels (gfx950).
//
// Distances are uint32 with INF = 2^31-1.  Every stored value is <= INF, so
// the sum of two of them is <= 2^32-2 and never wraps; min() with a stored
// value brings it back to <= INF.  That is the whole saturation scheme: one
// add and one min per relaxation, and results are exact for every distance
// below INF.
//
// Workgroups have 256 threads arranged as a 16x16 grid (tx = tid & 15,
// ty = tid >> 4).  A T x T tile (T = 64 or 128) is held in registers: thread
// (ty, tx) owns rows h*64 + ty*4 + a and columns h*64 + tx*4 + a for h < T/64,
// a < 4, i.e. an (T/16) x (T/16) block c[][].  Four consecutive columns are
// one 16-byte load or store, so a wave touches 4 rows x 256 contiguous bytes.
//
// All matrices are symmetric (undirected graphs), and the routines rely on
// it: column k of a tile is read as row k.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spq {

typedef uint32_t u32;
constexpr u32 INF = 0x7fffffffu;

__device__ __forceinline__ int tid_x() { return threadIdx.x & 15; }
__device__ __forceinline__ int tid_y() { return threadIdx.x >> 4; }

// min(a, b, c) as one v_min3_u32.  Written out because the compiler
// reassociates chains of min() into balanced trees (one v_min3 and two
// v_min for four candidates), which costs a third more VALU work.
__device__ __forceinline__ u32 min3u(u32 a, u32 b, u32 c) {
  u32 r;
  asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// c = min(c, a0 + b0, a1 + b1): two relaxations as v_add_u32, v_add_u32,
// v_min3_u32 in one asm statement.  The compiler cannot see into the
// statement and separates consecutive ones with an s_nop 0; the same three
// instructions issued back to back (what it emits from plain code) relax
// about a quarter slower on gfx950 (25.9 against 33.8 Trelax/s in a loop on
// LDS operands, 2,048 workgroups), and with a longer s_nop the gain is gone.
// The sums never wrap: all values are <= INF.
__device__ __forceinline__ void relax2(u32& c, u32 a0, u32 b0, u32 a1, u32 b1) {
  u32 t0, t1;
  asm volatile(
      "v_add_u32 %1, %3, %4\n\t"
      "v_add_u32 %2, %5, %6\n\t"
      "v_min3_u32 %0, %0, %1, %2"
      : "+v"(c), "=&v"(t0), "=&v"(t1)
      : "v"(a0), "v"(b0), "v"(a1), "v"(b1));
}

template <int T>
__device__ __forceinline__ void tile_load(u32 (&c)[T / 16][T / 16], const u32* __restrict__ g,
                                          int64_t ld) {
  const int tx = tid_x(), ty = tid_y();
#pragma unroll
  for (int h = 0; h < T / 64; h++)
#pragma unroll
    for (int a = 0; a < 4; a++) {
      const u32* row = g + (int64_t)(h * 64 + ty * 4 + a) * ld + tx * 4;
#pragma unroll
      for (int h2 = 0; h2 < T / 64; h2++) {
        uint4 v = *reinterpret_cast<const uint4*>(row + h2 * 64);
        c[h * 4 + a][h2 * 4 + 0] = v.x;
        c[h * 4 + a][h2 * 4 + 1] = v.y;
        c[h * 4 + a][h2 * 4 + 2] = v.z;
        c[h * 4 + a][h2 * 4 + 3] = v.w;
      }
    }
}

template <int T>
__device__ __forceinline__ void tile_store(const u32 (&c)[T / 16][T / 16], u32* __restrict__ g,
                                           int64_t ld) {
  const int tx = tid_x(), ty = tid_y();
#pragma unroll
  for (int h = 0; h < T / 64; h++)
#pragma unroll
    for (int a = 0; a < 4; a++) {
      u32* row = g + (int64_t)(h * 64 + ty * 4 + a) * ld + tx * 4;
#pragma unroll
      for (int h2 = 0; h2 < T / 64; h2++) {
        uint4 v = make_uint4(c[h * 4 + a][h2 * 4 + 0], c[h * 4 + a][h2 * 4 + 1],
                             c[h * 4 + a][h2 * 4 + 2], c[h * 4 + a][h2 * 4 + 3]);
        *reinterpret_cast<uint4*>(row + h2 * 64) = v;
      }
    }
}

// Stores the transpose: element (row x, col y) of the register tile goes to
// (row y, col x) of g.
template <int T>
__device__ __forceinline__ void tile_store_t(const u32 (&c)[T / 16][T / 16], u32* __restrict__ g,
                                             int64_t ld) {
  const int tx = tid_x(), ty = tid_y();
#pragma unroll
  for (int h2 = 0; h2 < T / 64; h2++)
#pragma unroll
    for (int a2 = 0; a2 < 4; a2++) {
      u32* row = g + (int64_t)(h2 * 64 + tx * 4 + a2) * ld + ty * 4;
#pragma unroll
      for (int h = 0; h < T / 64; h++) {
        uint4 v = make_uint4(c[h * 4 + 0][h2 * 4 + a2], c[h * 4 + 1][h2 * 4 + a2],
                             c[h * 4 + 2][h2 * 4 + a2], c[h * 4 + 3][h2 * 4 + a2]);
        *reinterpret_cast<uint4*>(row + h * 64) = v;
      }
    }
}

// Register tile -> LDS tile (row-major, row length T).
template <int T>
__device__ __forceinline__ void tile_to_lds(const u32 (&c)[T / 16][T / 16], u32* s) {
  const int tx = tid_x(), ty = tid_y();
#pragma unroll
  for (int h = 0; h < T / 64; h++)
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int h2 = 0; h2 < T / 64; h2++) {
        uint4 v = make_uint4(c[h * 4 + a][h2 * 4 + 0], c[h * 4 + a][h2 * 4 + 1],
                             c[h * 4 + a][h2 * 4 + 2], c[h * 4 + a][h2 * 4 + 3]);
        *reinterpret_cast<uint4*>(s + (h * 64 + ty * 4 + a) * T + h2 * 64 + tx * 4) = v;
      }
}

// c[i][j] = min(c[i][j], min over k < K of A[i][k] + B[k][j]), where the LDS
// arrays hold At[k][i] = A[i][k] and B[k][j], both with row length T.  The k
// order is free (a min-plus product), so two k are folded into one
// v_min3_u32: 1.5 VALU operations per relaxation.  K is even.
// NR: the thread's first NR rows only (NR = T/16 all of them; 4 with
// 128-tiles: the rows of the tile's first half); NC likewise for columns.
template <int T, int NR = T / 16, int NC = T / 16>
__device__ __forceinline__ void minplus_lds(u32 (&c)[T / 16][T / 16], const u32* At, const u32* B,
                                            int K) {
  constexpr int R = T / 16;
  const int tx = tid_x(), ty = tid_y();
  const u32* ap = At + ty * 4;
  const u32* bp = B + tx * 4;
#ifndef SPQ_MP_UNROLL
#define SPQ_MP_UNROLL 2
#endif
#pragma unroll SPQ_MP_UNROLL
  for (int k = 0; k < K; k += 2) {
    u32 a0[R], a1[R], b0[R], b1[R];
#pragma unroll
    for (int h = 0; h < T / 64; h++) {
      if (h * 4 < NR) {
        uint4 x0 = *reinterpret_cast<const uint4*>(ap + k * T + h * 64);
        uint4 x1 = *reinterpret_cast<const uint4*>(ap + (k + 1) * T + h * 64);
        a0[h * 4 + 0] = x0.x; a0[h * 4 + 1] = x0.y; a0[h * 4 + 2] = x0.z; a0[h * 4 + 3] = x0.w;
        a1[h * 4 + 0] = x1.x; a1[h * 4 + 1] = x1.y; a1[h * 4 + 2] = x1.z; a1[h * 4 + 3] = x1.w;
      }
      if (h * 4 < NC) {
        uint4 y0 = *reinterpret_cast<const uint4*>(bp + k * T + h * 64);
        uint4 y1 = *reinterpret_cast<const uint4*>(bp + (k + 1) * T + h * 64);
        b0[h * 4 + 0] = y0.x; b0[h * 4 + 1] = y0.y; b0[h * 4 + 2] = y0.z; b0[h * 4 + 3] = y0.w;
        b1[h * 4 + 0] = y1.x; b1[h * 4 + 1] = y1.y; b1[h * 4 + 2] = y1.z; b1[h * 4 + 3] = y1.w;
      }
    }
#pragma unroll
    for (int i = 0; i < NR; i++)
#pragma unroll
      for (int j = 0; j < NC; j++) relax2(c[i][j], a0[i], b0[j], a1[i], b1[j]);
  }
}

// Floyd-Warshall closure of the register tile (a symmetric matrix with a zero
// diagonal), pivots k = 0 .. T-1 in order.  Two pivots are taken per step:
// rows k and k+1 are published through LDS (double buffered, one barrier per
// step), row k+1 is first relaxed through pivot k, and then
//   c[i][j] = min(c[i][j], M[i][k] + M[k][j], M'[i][k+1] + M'[k+1][j])
// which is exactly pivot k followed by pivot k+1.  rb holds 4*T words.
template <int T>
__device__ __forceinline__ void fw_tile(u32 (&c)[T / 16][T / 16], u32* rb) {
  constexpr int R = T / 16;
  const int tx = tid_x(), ty = tid_y();
  for (int k = 0; k < T; k += 2) {
    u32* buf = rb + ((k >> 1) & 1) * 2 * T;
    const int owner = (k & 63) >> 2;          // ty owning rows k, k+1
    const int sel = ((k >> 6) << 2) | (k & 3); // their index in c[] (even)
    if (ty == owner) {
#pragma unroll
      for (int ii = 0; ii < R; ii += 2) {
        if (ii == sel) {
#pragma unroll
          for (int h2 = 0; h2 < T / 64; h2++) {
            *reinterpret_cast<uint4*>(buf + h2 * 64 + tx * 4) =
                make_uint4(c[ii][h2 * 4 + 0], c[ii][h2 * 4 + 1], c[ii][h2 * 4 + 2], c[ii][h2 * 4 + 3]);
            *reinterpret_cast<uint4*>(buf + T + h2 * 64 + tx * 4) =
                make_uint4(c[ii + 1][h2 * 4 + 0], c[ii + 1][h2 * 4 + 1], c[ii + 1][h2 * 4 + 2],
                           c[ii + 1][h2 * 4 + 3]);
          }
        }
      }
    }
    __syncthreads();
    const u32 s = buf[T + k];  // M[k+1][k]
    u32 rkc[R], rk1c[R], rkr[R], rk1r[R];
#pragma unroll
    for (int h = 0; h < T / 64; h++) {
      uint4 x = *reinterpret_cast<const uint4*>(buf + h * 64 + tx * 4);
      uint4 y = *reinterpret_cast<const uint4*>(buf + T + h * 64 + tx * 4);
      uint4 p = *reinterpret_cast<const uint4*>(buf + h * 64 + ty * 4);
      uint4 q = *reinterpret_cast<const uint4*>(buf + T + h * 64 + ty * 4);
      rkc[h * 4 + 0] = x.x; rkc[h * 4 + 1] = x.y; rkc[h * 4 + 2] = x.z; rkc[h * 4 + 3] = x.w;
      rk1c[h * 4 + 0] = y.x; rk1c[h * 4 + 1] = y.y; rk1c[h * 4 + 2] = y.z; rk1c[h * 4 + 3] = y.w;
      rkr[h * 4 + 0] = p.x; rkr[h * 4 + 1] = p.y; rkr[h * 4 + 2] = p.z; rkr[h * 4 + 3] = p.w;
      rk1r[h * 4 + 0] = q.x; rk1r[h * 4 + 1] = q.y; rk1r[h * 4 + 2] = q.z; rk1r[h * 4 + 3] = q.w;
    }
#pragma unroll
    for (int x = 0; x < R; x++) {
      rk1c[x] = min(rk1c[x], s + rkc[x]);
      rk1r[x] = min(rk1r[x], s + rkr[x]);
    }
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
      for (int j = 0; j < R; j++) relax2(c[i][j], rkr[i], rkc[j], rk1r[i], rk1c[j]);
  }
  __syncthreads();
}

}  // namespace spq
