// Parity sectors of d = 8 states: the sums of |Re| + |Im| over the even and
// odd total-parity parts of a full d^L state (exactly zero when that part is),
// and the conversion between the full tensor and the parity-halved layout
// (n_{L-1} = 2 m + ((n_0 + .. + n_{L-2} + sigma) mod 2), m = 0..3 stored at
// sum_{r < L-1} n_r 8^r + m 8^(L-1)).  The total parity is the parity of the
// base-8 digit sum of the flat index.
#include "device_common.h"

namespace fock {

namespace {

constexpr int kPerThread = 8;

__global__ __launch_bounds__(kBlock) void k_sector_norms(const float2 *__restrict__ psi, uint32_t n,
                                                         double *__restrict__ partial) {
  __shared__ double red[4];
  const uint32_t b0 = (uint32_t)blockIdx.x * (kBlock * kPerThread) + threadIdx.x;
  float se = 0.f, so = 0.f;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const uint32_t i = b0 + (uint32_t)k * kBlock;
    if (i < n) {
      const float2 v = psi[i];
      const float w = fabsf(v.x) + fabsf(v.y);
      if (octal_digit_parity(i)) so += w;
      else se += w;
    }
  }
  const double de = block_sum_d((double)se, red);
  const double dodd = block_sum_d((double)so, red);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = de;
    partial[2 * blockIdx.x + 1] = dodd;
  }
}

__global__ __launch_bounds__(kBlock) void k_sector_pack(const float2 *__restrict__ full, float2 *__restrict__ half,
                                                        uint32_t nhalf, int shift, int sector) {
  const uint32_t c = (uint32_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= nhalf) return;
  const uint32_t low = c & ((1u << shift) - 1u), m = c >> shift;
  const uint32_t top = 2u * m + (uint32_t)((octal_digit_parity(low) + sector) & 1);
  half[c] = full[low + (top << shift)];
}

__global__ __launch_bounds__(kBlock) void k_sector_unpack(const float2 *__restrict__ half, float2 *__restrict__ full,
                                                          uint32_t nhalf, int shift, int sector) {
  const uint32_t c = (uint32_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= nhalf) return;
  const uint32_t low = c & ((1u << shift) - 1u), m = c >> shift;
  const uint32_t top = 2u * m + (uint32_t)((octal_digit_parity(low) + sector) & 1);
  full[low + (top << shift)] = half[c];
  full[low + ((top ^ 1u) << shift)] = make_float2(0.f, 0.f);
}

}  // namespace

int sector_norms_blocks(uint32_t n) { return (int)((n + kBlock * kPerThread - 1) / (kBlock * kPerThread)); }

int launch_sector_norms(const float2 *psi, uint32_t n, double *partial, hipStream_t s) {
  hipLaunchKernelGGL(k_sector_norms, dim3(sector_norms_blocks(n)), dim3(kBlock), 0, s, psi, n, partial);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_sector_convert(int L, int sector, bool to_half, const float2 *src, float2 *dst, hipStream_t s) {
  if (L < 2 || L > 10) return set_error(FOCK_ERR_UNSUPPORTED, "parity-halved layout needs 2 <= L <= 10 (L=%d)", L);
  if (sector != 0 && sector != 1) return set_error(FOCK_ERR_ARG, "sector %d not in {0, 1}", sector);
  const int shift = 3 * (L - 1);
  const uint32_t nhalf = 4u << shift;
  const int G = (int)((nhalf + kBlock - 1) / kBlock);
  if (to_half)
    hipLaunchKernelGGL(k_sector_pack, dim3(G), dim3(kBlock), 0, s, src, dst, nhalf, shift, sector);
  else
    hipLaunchKernelGGL(k_sector_unpack, dim3(G), dim3(kBlock), 0, s, src, dst, nhalf, shift, sector);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
