// Two-mode gates and their reverse step on the top pair (L-2, L-1) of the
// parity-halved layout (d = 8).
//
// The generators keep the total parity (Sec. II.B: hopping moves one boson
// between the modes, pairing creates or removes two), so a state of parity
// sigma stores only m = 0..3 of the top mode, n_{L-1} = 2 m + q with q = (n_0 +
// .. + n_{L-2} + sigma) mod 2.  For the pair (i, j) = (L-2, L-1) and a fixed
// lower index f (modes 0..L-3, parity p), a member (n_i, n_j) is stored iff
// n_i + n_j = p + sigma (mod 2), at f + n_i d^i + (n_j >> 1) d^j.  A conserved
// block s (n_i + n_j = s for hopping, n_i - n_j = s - (d-1) for pairing) has a
// fixed n_i + n_j parity, so it is either stored whole or absent.
//
// One thread owns one lower index f and, as in the full layout, one wave runs
// one group of blocks for 64 consecutive f (every member load of a wave is one
// contiguous 512-byte run).  Consecutive f alternate p, so each lane zeroes the
// absent blocks of its group and does not store them: the loads and stores of
// a lane only touch its own stored members.
#include <cstring>

#include "gate_kernels.h"

namespace fock {

namespace {

constexpr int kHD = 8;  // cutoff of the halved layout
constexpr int kHNG = direct_groups<kHD>();
static_assert(kHNG == 4, "one block group per wave");

template <int KIND>
__device__ __forceinline__ bool half_block_stored(int s, int ps) {
  return ((s + (KIND == KIND_DIFF ? 1 : 0) + ps) & 1) == 0;
}

template <int KIND>
__device__ __forceinline__ uint32_t half_member_off(int s, int a, uint32_t si, uint32_t sj) {
  return (uint32_t)a * si + (uint32_t)(blk_nj(KIND, kHD, s, a) >> 1) * sj;
}

template <int KIND, bool DAG, int G>
__device__ __forceinline__ void gate_group_half(const float2 *src, float2 *base, uint32_t si, uint32_t sj,
                                                const float2 *__restrict__ U, int ps) {
  constexpr int D = kHD;
  constexpr Groups<D, kHNG> P{};
  float2 v[D * D];
  int m = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s)
    if (P.grp[s] == G) {
      const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
      const bool ok = half_block_stored<KIND>(s, ps);
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) v[m + q] = ok ? src[half_member_off<KIND>(s, lo + q, si, sj)] : make_float2(0.f, 0.f);
      m += b;
    }
  m = 0;
  int off = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s) {
    const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
    if (P.grp[s] == G) {
      const bool ok = half_block_stored<KIND>(s, ps);
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 o = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) {
              if (DAG) cmac_conj(o, U[off + q * b + p], v[m + q]);
              else cmac(o, U[off + p * b + q], v[m + q]);
            }
          if (ok) base[half_member_off<KIND>(s, lo + p, si, sj)] = o;
        }
      m += b;
    }
    off += b * b;
  }
}

// Reverse step on group G: sum Re(conj(lam) A phi) over the stored members,
// then phi <- U^+ phi (when WPHI) and lam <- U^+ lam on them.
template <int KIND, int G, bool WPHI>
__device__ __forceinline__ float adj_group_half(float2 *pb, float2 *lb, uint32_t si, uint32_t sj,
                                                const float2 *__restrict__ U, const float2 *__restrict__ A, int ps) {
  constexpr int D = kHD;
  constexpr Groups<D, kHNG> P{};
  float2 pv[D * D], lv[D * D];
  int m = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s)
    if (P.grp[s] == G) {
      const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
      const bool ok = half_block_stored<KIND>(s, ps);
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) {
          const uint32_t o = half_member_off<KIND>(s, lo + q, si, sj);
          pv[m + q] = ok ? pb[o] : make_float2(0.f, 0.f);
          lv[m + q] = ok ? lb[o] : make_float2(0.f, 0.f);
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
      const bool ok = half_block_stored<KIND>(s, ps);
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 ap = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b && q >= p - 1 && q <= p + 1) cmac(ap, A[off + p * b + q], pv[m + q]);
          gacc = fmaf(lv[m + p].x, ap.x, fmaf(lv[m + p].y, ap.y, gacc));
        }
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 np = make_float2(0.f, 0.f), nl = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) {
              const float2 u = U[off + q * b + p];
              if (WPHI) cmac_conj(np, u, pv[m + q]);
              cmac_conj(nl, u, lv[m + q]);
            }
          if (ok) {
            const uint32_t o = half_member_off<KIND>(s, lo + p, si, sj);
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

// GateLaunch of the top pair: nfib = d^(L-2) lower indices, si = d^(L-2),
// sj = d^(L-1); the lower index f is also the fiber's base offset.
template <int KIND, bool DAG>
__global__ __launch_bounds__(kBlock) void k_gate2_half(const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                                       GateLaunch g, int sector) {
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t f = (uint32_t)vb * 64 + lane;
  if (f >= g.nfib) return;
  const int ps = (octal_digit_parity(f) + sector) & 1;
  const float2 *sb = src + f;
  float2 *base = psi + f;
  switch (wave) {
    case 0: gate_group_half<KIND, DAG, 0>(sb, base, g.si, g.sj, U, ps); break;
    case 1: gate_group_half<KIND, DAG, 1>(sb, base, g.si, g.sj, U, ps); break;
    case 2: gate_group_half<KIND, DAG, 2>(sb, base, g.si, g.sj, U, ps); break;
    default: gate_group_half<KIND, DAG, 3>(sb, base, g.si, g.sj, U, ps); break;
  }
}

template <int KIND, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_gate2_adj_half(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                           const float2 *__restrict__ U, const float2 *__restrict__ A,
                                                           double *__restrict__ partial, GateLaunch g, int sector) {
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t f = (uint32_t)vb * 64 + lane;
  float gacc = 0.f;
  if (f < g.nfib) {
    const int ps = (octal_digit_parity(f) + sector) & 1;
    float2 *pb = phi + f, *lb = lam + f;
    switch (wave) {
      case 0: gacc = adj_group_half<KIND, 0, WPHI>(pb, lb, g.si, g.sj, U, A, ps); break;
      case 1: gacc = adj_group_half<KIND, 1, WPHI>(pb, lb, g.si, g.sj, U, A, ps); break;
      case 2: gacc = adj_group_half<KIND, 2, WPHI>(pb, lb, g.si, g.sj, U, A, ps); break;
      default: gacc = adj_group_half<KIND, 3, WPHI>(pb, lb, g.si, g.sj, U, A, ps); break;
    }
  }
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

GateLaunch half_top_launch(const Geometry &g) {
  GateLaunch gl;
  memset(&gl, 0, sizeof(gl));
  uint32_t si = 1;
  for (int r = 0; r < g.L - 2; ++r) si *= (uint32_t)kHD;
  gl.si = si;
  gl.sj = si * (uint32_t)kHD;
  gl.nfib = si;
  return gl;
}

int check_half_top(const Geometry &g, int i, int j) {
  if (!g.half || g.d != kHD || g.L < 3 || g.L > 10 || i != g.L - 2 || j != g.L - 1)
    return set_error(FOCK_ERR_UNSUPPORTED, "pair (%d,%d) in the parity-halved layout of L=%d, d=%d", i, j, g.L, g.d);
  if (g.n_amp != half_top_launch(g).sj / 2 * (uint32_t)kHD)
    return set_error(FOCK_ERR_SIZE, "parity-halved state of %u amplitudes", g.n_amp);
  return FOCK_OK;
}

}  // namespace

int half_top_blocks(const Geometry &g) { return (int)((half_top_launch(g).nfib + 63) / 64); }

int launch_gate_half(const Geometry &g, int i, int j, int kind, bool dag, const float2 *U, const float2 *src,
                     float2 *psi, hipStream_t s) {
  int rc = check_half_top(g, i, j);
  if (rc) return rc;
  const GateLaunch gl = half_top_launch(g);
  const int G = half_top_blocks(g);
#define GH(K, DG) hipLaunchKernelGGL((k_gate2_half<K, DG>), dim3(G), dim3(kBlock), 0, s, src, psi, U, gl, g.sector)
  if (kind == KIND_SUM) {
    if (dag) GH(KIND_SUM, true); else GH(KIND_SUM, false);
  } else {
    if (dag) GH(KIND_DIFF, true); else GH(KIND_DIFF, false);
  }
#undef GH
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_gate_adj_half(const Geometry &g, int i, int j, int kind, const float2 *U, const float2 *A, float2 *phi,
                         float2 *lam, double *partial, hipStream_t s, bool write_phi) {
  int rc = check_half_top(g, i, j);
  if (rc) return rc;
  const GateLaunch gl = half_top_launch(g);
  const int G = half_top_blocks(g);
#define AH(K, W)                                                                                             \
  hipLaunchKernelGGL((k_gate2_adj_half<K, W>), dim3(G), dim3(kBlock), 0, s, phi, lam, U, A, partial, gl, \
                     g.sector)
  if (kind == KIND_SUM) {
    if (write_phi) AH(KIND_SUM, true); else AH(KIND_SUM, false);
  } else {
    if (write_phi) AH(KIND_DIFF, true); else AH(KIND_DIFF, false);
  }
#undef AH
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
