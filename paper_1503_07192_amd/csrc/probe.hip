// Issue rates of the VALU instructions the min-plus kernels are made of,
// measured on the device.  They fix the relaxation peak the kernels are
// compared with: a relaxation is one v_add_u32 and half a v_min3_u32 (two
// candidates per min3), so the peak is set by how many of each a CU issues
// per clock.
//   kind 0: v_add_u32 only    kind 1: v_min3_u32 only
//   (eight chains per lane, each four dependent instructions per iteration,
//   emitted chain after chain: a wave waits on its own results and the
//   other waves of the SIMD fill the gaps)
//   kind 2: the production relaxation loop (minplus_lds of tiles.h) on LDS
//   operands, no global memory inside the loop
//   kind 3: the same relaxation pairs (relax2) on operands held in registers:
//   no LDS reads either, so the loop is the instruction sequence alone
#include "spq_internal.h"
#include "tiles.h"

namespace spq {

template <int OP>
__global__ __launch_bounds__(256) void k_rate(u32* __restrict__ out, int iters, u32 seed) {
  u32 x[8], y = seed ^ threadIdx.x, z = seed + blockIdx.x;
#pragma unroll
  for (int i = 0; i < 8; i++) x[i] = threadIdx.x * 7u + i;
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (OP == 0) {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[i]) : "v"(y));
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[i]) : "v"(z));
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[i]) : "v"(y));
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[i]) : "v"(z));
      } else {
        asm volatile("v_min3_u32 %0, %0, %1, %2" : "+v"(x[i]) : "v"(y), "v"(z));
        asm volatile("v_min3_u32 %0, %0, %1, %2" : "+v"(x[i]) : "v"(z), "v"(y));
        asm volatile("v_min3_u32 %0, %0, %1, %2" : "+v"(x[i]) : "v"(y), "v"(z));
        asm volatile("v_min3_u32 %0, %0, %1, %2" : "+v"(x[i]) : "v"(z), "v"(y));
      }
    }
  }
  u32 s = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) s += x[i];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_rate_relax(u32* __restrict__ out, int iters, u32 seed) {
  __shared__ __attribute__((aligned(16))) u32 sA[16 * 128];
  __shared__ __attribute__((aligned(16))) u32 sB[16 * 128];
  for (int e = threadIdx.x; e < 16 * 128; e += 256) {
    sA[e] = (e * 2654435761u + seed) >> 4;
    sB[e] = (e * 40503u + seed * 7u) >> 4;
  }
  __syncthreads();
  u32 c[8][8];
#pragma unroll
  for (int i = 0; i < 8; i++)
#pragma unroll
    for (int j = 0; j < 8; j++) c[i][j] = INF - (u32)(i + j) - threadIdx.x;
  for (int it = 0; it < iters; it++) minplus_lds<128>(c, sA, sB, 16);
  u32 s = 0;
#pragma unroll
  for (int i = 0; i < 8; i++)
#pragma unroll
    for (int j = 0; j < 8; j++) s ^= c[i][j];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_rate_relax_regs(u32* __restrict__ out, int iters, u32 seed) {
  u32 a0[8], b0[8], a1[8], b1[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    a0[i] = ((threadIdx.x + i) * 2654435761u + seed) >> 4;
    b0[i] = ((threadIdx.x + 3 * i) * 40503u + seed) >> 4;
    a1[i] = ((threadIdx.x + 5 * i) * 2246822519u + seed) >> 4;
    b1[i] = ((threadIdx.x + 7 * i) * 3266489917u + seed) >> 4;
  }
  u32 c[8][8];
#pragma unroll
  for (int i = 0; i < 8; i++)
#pragma unroll
    for (int j = 0; j < 8; j++) c[i][j] = INF - (u32)(i + j) - threadIdx.x;
  // eight pairs of k per iteration: the relaxations of one 16-row chunk
  for (int it = 0; it < iters; it++)
    for (int kk = 0; kk < 8; kk++)
#pragma unroll
      for (int i = 0; i < 8; i++)
#pragma unroll
        for (int j = 0; j < 8; j++) relax2(c[i][j], a0[i], b0[j], a1[i], b1[j]);
  u32 s = 0;
#pragma unroll
  for (int i = 0; i < 8; i++)
#pragma unroll
    for (int j = 0; j < 8; j++) s ^= c[i][j];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// out: blocks * 256 words.  Work per launch: kinds 0/1: blocks * 256 lanes *
// iters * 32 instructions; kinds 2/3: blocks * 256 * 64 * 16 * iters relaxations.
hipError_t launch_valu_probe(int kind, int blocks, int iters, u32* out, hipStream_t s) {
  if (kind == 0)
    k_rate<0><<<blocks, 256, 0, s>>>(out, iters, 2u);
  else if (kind == 1)
    k_rate<1><<<blocks, 256, 0, s>>>(out, iters, 2u);
  else if (kind == 2)
    k_rate_relax<<<blocks, 256, 0, s>>>(out, iters, 2u);
  else
    k_rate_relax_regs<<<blocks, 256, 0, s>>>(out, iters, 2u);
  return hipGetLastError();
}

}  // namespace spq
