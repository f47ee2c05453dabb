// Per-fiber block arithmetic of the real gates HR, PR (d = 8) on float32
// amplitudes: the conserved-block groups of one fiber mapped through U or U^T,
// and the reverse step's gradient term.  Shared by the per-gate kernels
// (gate_real.hip) and the fused runs (gate_real_fuse.hip); member addresses are
// a * si + n_j * sj from a fiber base in global memory or in an LDS tile.
#pragma once

#include "gate_kernels.h"

namespace fock {
namespace rgates {

constexpr int kRD = 8;
constexpr int kRNG = direct_groups<kRD>();
static_assert(kRNG == 4, "one block group per wave");

// Member offsets of the top pair of the parity-halved layout (see gate_half.hip).
template <int KIND>
__device__ __forceinline__ bool rhalf_stored(int s, int ps) {
  return ((s + (KIND == KIND_DIFF ? 1 : 0) + ps) & 1) == 0;
}

template <int KIND, bool HALF>
__device__ __forceinline__ uint32_t rmember(int s, int a, uint32_t si, uint32_t sj) {
  const int nj = blk_nj(KIND, kRD, s, a);
  return (uint32_t)a * si + (uint32_t)(HALF ? (nj >> 1) : nj) * sj;
}

// psi <- U src (U^T src when DAG) on group G of one fiber; HALF: the top pair
// of the parity-halved layout, ps = lower modes' parity plus the sector.  UP
// reads the packed table: a global pointer, or a table staged in LDS.
template <int KIND, bool DAG, int G, bool HALF, class UP = const float2 *__restrict__, int PS = -1>
__device__ __forceinline__ void rgate_group(const float *src, float *base, uint32_t si, uint32_t sj, UP U, int ps) {
  if (PS >= 0) ps = PS;  // a compile-time parity drops the absent blocks' code
  constexpr int D = kRD;
  constexpr Groups<D, kRNG> P{};
  float v[D * D];
  int m = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s)
    if (P.grp[s] == G) {
      const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
      const bool ok = !HALF || rhalf_stored<KIND>(s, ps);
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) v[m + q] = ok ? src[rmember<KIND, HALF>(s, lo + q, si, sj)] : 0.f;
      m += b;
    }
  m = 0;
  int off = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s) {
    const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
    if (P.grp[s] == G) {
      const bool ok = !HALF || rhalf_stored<KIND>(s, ps);
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float o = 0.f;
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) o = fmaf(DAG ? U[off + q * b + p].x : U[off + p * b + q].x, v[m + q], o);
          if (ok) base[rmember<KIND, HALF>(s, lo + p, si, sj)] = o;
        }
      m += b;
    }
    off += b * b;
  }
}

// Reverse step on group G: sum lam . (A phi) over the group's members, then
// phi <- U^T phi (when WPHI) and lam <- U^T lam.
template <int KIND, int G, bool WPHI, bool HALF, class UP = const float2 *__restrict__, int PS = -1>
__device__ __forceinline__ float radj_group(float *pb, float *lb, uint32_t si, uint32_t sj, UP U, UP A, int ps) {
  if (PS >= 0) ps = PS;
  constexpr int D = kRD;
  constexpr Groups<D, kRNG> P{};
  float pv[D * D], lv[D * D];
  int m = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s)
    if (P.grp[s] == G) {
      const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
      const bool ok = !HALF || rhalf_stored<KIND>(s, ps);
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) {
          const uint32_t o = rmember<KIND, HALF>(s, lo + q, si, sj);
          pv[m + q] = ok ? pb[o] : 0.f;
          lv[m + q] = ok ? lb[o] : 0.f;
        }
      m += b;
    }
  float gacc = 0.f;
  m = 0;
  int off = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s) {
    const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
    if (P.grp[s] == G) {
      const bool ok = !HALF || rhalf_stored<KIND>(s, ps);
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float ap = 0.f;
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b && q >= p - 1 && q <= p + 1) ap = fmaf(A[off + p * b + q].x, pv[m + q], ap);
          gacc = fmaf(lv[m + p], ap, gacc);
        }
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float np = 0.f, nl = 0.f;
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) {
              const float u = U[off + q * b + p].x;
              if (WPHI) np = fmaf(u, pv[m + q], np);
              nl = fmaf(u, lv[m + q], nl);
            }
          if (ok) {
            const uint32_t o = rmember<KIND, HALF>(s, lo + p, si, sj);
            if (WPHI) pb[o] = np;
            lb[o] = nl;
          }
        }
      m += b;
    }
    off += b * b;
  }
  return gacc;
}

}  // namespace rgates
}  // namespace fock
