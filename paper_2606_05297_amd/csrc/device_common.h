// Device helpers shared by the HIP kernels (gfx950, wave64).
#pragma once

#include "fock_internal.h"

namespace fock {

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Remap so that XCD x processes a contiguous run of virtual blocks:
// neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7) * q + (b >> 3);
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread workgroup in double; result valid in thread 0.
__device__ __forceinline__ double block_sum_d(double v, double *lds4) {
  v = wave_sum_d(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds4[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
  __syncthreads();
  return r;
}

template <int D>
__device__ __forceinline__ void load_row(const float2 *__restrict__ p, float2 (&v)[D]) {
  if constexpr (D % 2 == 0) {
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int k = 0; k < D / 2; ++k) {
      const float4 t = q[k];
      v[2 * k] = make_float2(t.x, t.y);
      v[2 * k + 1] = make_float2(t.z, t.w);
    }
  } else {
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = p[k];
  }
}

template <int D>
__device__ __forceinline__ void store_row(float2 *__restrict__ p, const float2 (&v)[D]) {
  if constexpr (D % 2 == 0) {
    float4 *q = reinterpret_cast<float4 *>(p);
#pragma unroll
    for (int k = 0; k < D / 2; ++k) q[k] = make_float4(v[2 * k].x, v[2 * k].y, v[2 * k + 1].x, v[2 * k + 1].y);
  } else {
#pragma unroll
    for (int k = 0; k < D; ++k) p[k] = v[k];
  }
}

// acc += c * row
template <int D>
__device__ __forceinline__ void axpy_row(float2 (&acc)[D], const float2 *__restrict__ p, float c) {
  float2 v[D];
  load_row<D>(p, v);
#pragma unroll
  for (int q = 0; q < D; ++q) {
    acc[q].x = fmaf(c, v[q].x, acc[q].x);
    acc[q].y = fmaf(c, v[q].y, acc[q].y);
  }
}

__host__ __device__ constexpr int blk_lo(int kind, int d, int s) {
  return kind == KIND_SUM ? (s - (d - 1) > 0 ? s - (d - 1) : 0) : (s - (d - 1) > 0 ? s - (d - 1) : 0);
}
__host__ __device__ constexpr int blk_hi(int kind, int d, int s) {
  return kind == KIND_SUM ? (s < d - 1 ? s : d - 1) : (s < d - 1 ? s : d - 1);
}
// n_j of member a in block s.
__host__ __device__ constexpr int blk_nj(int kind, int d, int s, int a) {
  return kind == KIND_SUM ? s - a : a - (s - (d - 1));
}

}  // namespace fock
