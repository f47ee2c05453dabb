// Gate kernels (templated on the cutoff d); instantiated per d in the
// kernels_gate_d*.hip translation units so they compile in parallel.
#pragma once

#include "device_common.h"

namespace fock {

struct GateLaunch {
  uint32_t nfib, si, sj;
  FastDiv dsi, dm1;
};
// Launch parameters of a gate on (i, j) in geometry g (kernels_gate.hip).
GateLaunch gate_launch_params(const Geometry &g, int i, int j);

__device__ __forceinline__ uint32_t fiber_base(uint32_t f, const GateLaunch &g, int D) {
  const uint32_t t = fdiv(f, g.dsi);
  const uint32_t low = f - t * g.si;
  const uint32_t high = fdiv(t, g.dm1);
  const uint32_t mid = t - high * g.dm1.v;
  return low + mid * g.si * (uint32_t)D + high * g.sj * (uint32_t)D;
}

__device__ __forceinline__ void cmac(float2 &o, float2 u, float2 v) {
  o.x = fmaf(u.x, v.x, fmaf(-u.y, v.y, o.x));
  o.y = fmaf(u.x, v.y, fmaf(u.y, v.x, o.y));
}
// o += conj(u) * v
__device__ __forceinline__ void cmac_conj(float2 &o, float2 u, float2 v) {
  o.x = fmaf(u.x, v.x, fmaf(u.y, v.y, o.x));
  o.y = fmaf(u.x, v.y, fmaf(-u.y, v.x, o.y));
}

// ---------------------------------------------------------------- block groups
// The 2d-1 conserved blocks of a fiber are split into NG groups of nearly
// equal size (greedy, largest block first).  One wavefront handles one group
// for 64 fibers, so every lane of a wave runs the same compile-time block
// code (no divergence) and the gate matrix entries are wave-uniform.
template <int D, int NG>
struct Groups {
  static constexpr int NB = 2 * D - 1;
  int grp[NB];
  int size[NG];
  constexpr Groups() : grp(), size() {
    for (int k = 0; k < NB; ++k) grp[k] = 0;
    for (int g = 0; g < NG; ++g) size[g] = 0;
    // blocks in order of decreasing size: s = D-1, D-2, D, D-3, D+1, ...
    for (int k = 0; k < NB; ++k) {
      const int s = (k == 0) ? D - 1 : ((k & 1) ? D - 1 - (k + 1) / 2 : D - 1 + k / 2);
      const int b = (s < D - 1 ? s : 2 * D - 2 - s) + 1;
      int best = 0;
      for (int g = 1; g < NG; ++g)
        if (size[g] < size[best]) best = g;
      grp[s] = best;
      size[best] += b;
    }
  }
};

template <int D>
constexpr int direct_groups() { return D <= 3 ? 1 : (D <= 6 ? 2 : 4); }

template <int D, int KIND>
__device__ __forceinline__ uint32_t member_off(int s, int a, uint32_t si, uint32_t sj) {
  return (uint32_t)a * si + (uint32_t)blk_nj(KIND, D, s, a) * sj;
}

// Apply U (or U^+) to the members of group G of one fiber.  ld/st address the
// member (s, a): global memory (direct) or an LDS tile (mode-0 pairs).
template <int D, int KIND, bool DAG, int NG, int G, class Ptr, class CPtr>
__device__ __forceinline__ void gate_group_blockwise(CPtr src, Ptr base, uint32_t si, uint32_t sj,
                                                     const float2 *__restrict__ U) {
  constexpr Groups<D, NG> P{};
  int off = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s) {
    const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
    if (P.grp[s] == G) {
      float2 v[D];
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) v[q] = src[member_off<D, KIND>(s, lo + q, si, sj)];
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 o = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) {
              if (DAG) cmac_conj(o, U[off + q * b + p], v[q]);
              else cmac(o, U[off + p * b + q], v[q]);
            }
          base[member_off<D, KIND>(s, lo + p, si, sj)] = o;
        }
    }
    off += b * b;
  }
}

// src: members are read there; base: results are written there (src == base
// for the in-place gate).
template <int D, int KIND, bool DAG, int NG, int G, class Ptr, class CPtr>
__device__ __forceinline__ void gate_group(CPtr src, Ptr base, uint32_t si, uint32_t sj, const float2 *__restrict__ U) {
  if constexpr (D > 8) {
    gate_group_blockwise<D, KIND, DAG, NG, G>(src, base, si, sj, U);
    return;
  }
  constexpr Groups<D, NG> P{};
  float2 v[D * D];
  int m = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s)
    if (P.grp[s] == G) {
      const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) v[m + q] = src[member_off<D, KIND>(s, lo + q, si, sj)];
      m += b;
    }
  m = 0;
  int off = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s) {
    const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
    if (P.grp[s] == G) {
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
          base[member_off<D, KIND>(s, lo + p, si, sj)] = o;
        }
      m += b;
    }
    off += b * b;
  }
}

// Fused reverse step on group G: returns sum Re(conj(lam) A phi) over the
// group's members, then phi <- U^+ phi (only when WPHI: with the forward
// states kept, phi is read-only), lam <- U^+ lam.  A's blocks are tridiagonal
// in the member order (the generators move n_i by one).
template <int D, int KIND, int NG, int G, bool WPHI = true, class Ptr>
__device__ __forceinline__ float adj_group_blockwise(Ptr pb, Ptr lb, uint32_t si, uint32_t sj,
                                                     const float2 *__restrict__ U, const float2 *__restrict__ A) {
  constexpr Groups<D, NG> P{};
  float gacc = 0.f;
  int off = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s) {
    const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
    if (P.grp[s] == G) {
      float2 pv[D], lv[D];
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) {
          const uint32_t o = member_off<D, KIND>(s, lo + q, si, sj);
          pv[q] = pb[o];
          lv[q] = lb[o];
        }
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 ap = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b && q >= p - 1 && q <= p + 1) cmac(ap, A[off + p * b + q], pv[q]);
          gacc = fmaf(lv[p].x, ap.x, fmaf(lv[p].y, ap.y, gacc));
        }
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 np = make_float2(0.f, 0.f), nl = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) {
              const float2 u = U[off + q * b + p];
              if (WPHI) cmac_conj(np, u, pv[q]);
              cmac_conj(nl, u, lv[q]);
            }
          const uint32_t o = member_off<D, KIND>(s, lo + p, si, sj);
          if (WPHI) pb[o] = np;
          lb[o] = nl;
        }
    }
    off += b * b;
  }
  return gacc;
}

template <int D, int KIND, int NG, int G, bool WPHI = true, class Ptr>
__device__ __forceinline__ float adj_group(Ptr pb, Ptr lb, uint32_t si, uint32_t sj, const float2 *__restrict__ U,
                                           const float2 *__restrict__ A) {
  if constexpr (D > 8) return adj_group_blockwise<D, KIND, NG, G, WPHI>(pb, lb, si, sj, U, A);
  constexpr Groups<D, NG> P{};
  float2 pv[D * D], lv[D * D];
  int m = 0;
#pragma unroll
  for (int s = 0; s < 2 * D - 1; ++s)
    if (P.grp[s] == G) {
      const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) {
          const uint32_t o = member_off<D, KIND>(s, lo + q, si, sj);
          pv[m + q] = pb[o];
          lv[m + q] = lb[o];
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
          const uint32_t o = member_off<D, KIND>(s, lo + p, si, sj);
          if (WPHI) pb[o] = np;
          lb[o] = nl;
        }
      m += b;
    }
    off += b * b;
  }
  return gacc;
}

// ---------------------------------------------------------------- pairs (i, j) with i >= 1
// Consecutive lanes own fibers that differ in the lowest free mode (mode 0),
// so each member access of a wavefront is one contiguous 512-byte run.
// The *_block device functions do the work of workgroup vb; the kernels below
// and the batched sweep kernels call them.
template <int D, int KIND, bool DAG>
__device__ __forceinline__ void gate2_direct_block(int vb, const float2 *src, float2 *psi,
                                                   const float2 *__restrict__ U, const GateLaunch &g) {
  constexpr int NG = direct_groups<D>();
  constexpr int FPB = 64 * (4 / NG);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gi = wave % NG;
  const uint32_t f = (uint32_t)vb * FPB + (uint32_t)(wave / NG) * 64 + lane;
  if (f >= g.nfib) return;
  const uint32_t fb = fiber_base(f, g, D);
  const float2 *sb = src + fb;
  float2 *base = psi + fb;
  switch (gi) {
    case 0: gate_group<D, KIND, DAG, NG, 0>(sb, base, g.si, g.sj, U); break;
    case 1: if constexpr (NG > 1) gate_group<D, KIND, DAG, NG, 1>(sb, base, g.si, g.sj, U); break;
    case 2: if constexpr (NG > 2) gate_group<D, KIND, DAG, NG, 2>(sb, base, g.si, g.sj, U); break;
    default: if constexpr (NG > 3) gate_group<D, KIND, DAG, NG, 3>(sb, base, g.si, g.sj, U); break;
  }
}

template <int D, int KIND, bool WPHI = true>
__device__ __forceinline__ float adj_direct_block(int vb, float2 *phi, float2 *lam, const float2 *__restrict__ U,
                                                  const float2 *__restrict__ A, const GateLaunch &g) {
  constexpr int NG = direct_groups<D>();
  constexpr int FPB = 64 * (4 / NG);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gi = wave % NG;
  const uint32_t f = (uint32_t)vb * FPB + (uint32_t)(wave / NG) * 64 + lane;
  float gacc = 0.f;
  if (f < g.nfib) {
    const uint32_t fb = fiber_base(f, g, D);
    float2 *pb = phi + fb, *lb = lam + fb;
    switch (gi) {
      case 0: gacc = adj_group<D, KIND, NG, 0, WPHI>(pb, lb, g.si, g.sj, U, A); break;
      case 1: if constexpr (NG > 1) gacc = adj_group<D, KIND, NG, 1, WPHI>(pb, lb, g.si, g.sj, U, A); break;
      case 2: if constexpr (NG > 2) gacc = adj_group<D, KIND, NG, 2, WPHI>(pb, lb, g.si, g.sj, U, A); break;
      default: if constexpr (NG > 3) gacc = adj_group<D, KIND, NG, 3, WPHI>(pb, lb, g.si, g.sj, U, A); break;
    }
  }
  return gacc;
}

template <int D, int KIND, bool DAG>
__global__ __launch_bounds__(kBlock) void k_gate2(const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                                  GateLaunch g) {
  gate2_direct_block<D, KIND, DAG>(xcd_remap(blockIdx.x, gridDim.x), src, psi, U, g);
}

template <int D, int KIND, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_gate2_adj(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                      const float2 *__restrict__ U, const float2 *__restrict__ A,
                                                      double *__restrict__ partial, GateLaunch g) {
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const float gacc = adj_direct_block<D, KIND, WPHI>(vb, phi, lam, U, A, g);
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

// ---------------------------------------------------------------- pairs (0, j): LDS-staged
// Mode 0 is the contiguous one, so a fiber's members are runs of d amplitudes
// and thread-per-fiber access would scatter a wavefront over 64 runs.  The
// workgroup instead copies FL fibers into LDS with contiguous global accesses
// (lanes run along n_0, then along consecutive fibers), the four waves apply
// the four block groups from LDS, and the tile is copied back.
template <int D>
constexpr int lds_fibers() { return D * D <= 64 ? 64 : 16; }
// LDS floats (float2 units) of one fiber tile and of the fiber base table
template <int D>
constexpr int m0_tile_elems() { return lds_fibers<D>() * (D * D + 1); }

template <int D>
__device__ __forceinline__ void tile_copy(float2 *tile, float2 *gmem, const uint32_t *fbase, uint32_t sj,
                                          bool to_lds, uint32_t nf) {
  constexpr int FL = lds_fibers<D>(), ST = D * D + 1;
  if constexpr (D % 2 == 0) {
    // two consecutive n_0 values per access: 16-byte global loads/stores
    for (int e = threadIdx.x; e < FL * D * D / 2; e += kBlock) {
      const int b = e / (FL * D / 2), r = e % (FL * D / 2);
      const int fl = r / (D / 2), a = 2 * (r % (D / 2));
      if ((uint32_t)fl < nf) {
        const uint32_t gi = fbase[fl] + (uint32_t)a + (uint32_t)b * sj;
        float4 *gp = reinterpret_cast<float4 *>(gmem + gi);
        float2 *tp = tile + fl * ST + b * D + a;
        if (to_lds) {
          const float4 v = *gp;
          tp[0] = make_float2(v.x, v.y);
          tp[1] = make_float2(v.z, v.w);
        } else {
          *gp = make_float4(tp[0].x, tp[0].y, tp[1].x, tp[1].y);
        }
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < FL * D * D; e += kBlock) {
    const int b = e / (FL * D), r = e % (FL * D);
    const int fl = r / D, a = r % D;
    if ((uint32_t)fl < nf) {
      const uint32_t gi = fbase[fl] + (uint32_t)a + (uint32_t)b * sj;
      if (to_lds) tile[fl * ST + b * D + a] = gmem[gi];
      else gmem[gi] = tile[fl * ST + b * D + a];
    }
  }
}

// tile: m0_tile_elems<D>() float2 of LDS; fbase: lds_fibers<D>() words of LDS.
// Contains barriers: every thread of the workgroup must call it.
template <int D, int KIND, bool DAG>
__device__ __forceinline__ void gate2_m0_block(int vb, const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                               const GateLaunch &g, float2 *tile, uint32_t *fbase) {
  constexpr int FL = lds_fibers<D>(), ST = D * D + 1;
  const uint32_t f0 = (uint32_t)vb * FL;
  const uint32_t nf = g.nfib - f0 < (uint32_t)FL ? g.nfib - f0 : (uint32_t)FL;
  if (threadIdx.x < FL && threadIdx.x < nf) fbase[threadIdx.x] = fiber_base(f0 + threadIdx.x, g, D);
  __syncthreads();
  tile_copy<D>(tile, const_cast<float2 *>(src), fbase, g.sj, true, nf);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if ((uint32_t)lane < nf && lane < FL) {
    float2 *base = tile + lane * ST;
    // member (n_0 = a, n_j = b) sits at b * D + a in the fiber's LDS row
    switch (wave) {
      case 0: gate_group<D, KIND, DAG, 4, 0>(base, base, 1u, (uint32_t)D, U); break;
      case 1: gate_group<D, KIND, DAG, 4, 1>(base, base, 1u, (uint32_t)D, U); break;
      case 2: gate_group<D, KIND, DAG, 4, 2>(base, base, 1u, (uint32_t)D, U); break;
      default: gate_group<D, KIND, DAG, 4, 3>(base, base, 1u, (uint32_t)D, U); break;
    }
  }
  __syncthreads();
  tile_copy<D>(tile, psi, fbase, g.sj, false, nf);
  __syncthreads();
}

template <int D, int KIND, bool WPHI = true>
__device__ __forceinline__ float adj_m0_block(int vb, float2 *phi, float2 *lam, const float2 *__restrict__ U,
                                              const float2 *__restrict__ A, const GateLaunch &g, float2 *tp,
                                              float2 *tl, uint32_t *fbase) {
  constexpr int FL = lds_fibers<D>(), ST = D * D + 1;
  const uint32_t f0 = (uint32_t)vb * FL;
  const uint32_t nf = g.nfib - f0 < (uint32_t)FL ? g.nfib - f0 : (uint32_t)FL;
  if (threadIdx.x < FL && threadIdx.x < nf) fbase[threadIdx.x] = fiber_base(f0 + threadIdx.x, g, D);
  __syncthreads();
  tile_copy<D>(tp, phi, fbase, g.sj, true, nf);
  tile_copy<D>(tl, lam, fbase, g.sj, true, nf);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float gacc = 0.f;
  if ((uint32_t)lane < nf && lane < FL) {
    float2 *pb = tp + lane * ST, *lb = tl + lane * ST;
    switch (wave) {
      case 0: gacc = adj_group<D, KIND, 4, 0, WPHI>(pb, lb, 1u, (uint32_t)D, U, A); break;
      case 1: gacc = adj_group<D, KIND, 4, 1, WPHI>(pb, lb, 1u, (uint32_t)D, U, A); break;
      case 2: gacc = adj_group<D, KIND, 4, 2, WPHI>(pb, lb, 1u, (uint32_t)D, U, A); break;
      default: gacc = adj_group<D, KIND, 4, 3, WPHI>(pb, lb, 1u, (uint32_t)D, U, A); break;
    }
  }
  __syncthreads();
  if (WPHI) tile_copy<D>(tp, phi, fbase, g.sj, false, nf);
  tile_copy<D>(tl, lam, fbase, g.sj, false, nf);
  __syncthreads();
  return gacc;
}

// ---------------------------------------------------------------- pairs (0, j), d = 8: pipelined tiles
// A workgroup walks kM0Tiles consecutive 64-fibre tiles.  The next tile's
// global loads go out (into registers) before the current tile is computed in
// LDS and stored, so memory latency overlaps the compute and store phases
// instead of separating them.  Loads are issued before the current tile's
// stores, so waiting for them never waits for those stores.  Used when every
// workgroup has whole tiles (d = 8 and a fibre count divisible by 64 kM0Tiles).
constexpr int kM0Tiles = 4;

template <int D>
__device__ __forceinline__ void m0_bases(uint32_t tile, const GateLaunch &g, uint32_t *fb) {
  constexpr int FL = lds_fibers<D>();
  if (threadIdx.x < FL) fb[threadIdx.x] = fiber_base(tile * FL + threadIdx.x, g, D);
}

// Thread's share of a tile: PER float4 (two n_0 values each), rows b = i.
template <int D>
constexpr int m0_per_thread() { return lds_fibers<D>() * D * D / 2 / kBlock; }

template <int D>
__device__ __forceinline__ void m0_gload(const float2 *src, const uint32_t *fb, uint32_t sj,
                                         float4 (&buf)[m0_per_thread<D>()]) {
  constexpr int HALF = lds_fibers<D>() * D / 2;
#pragma unroll
  for (int i = 0; i < m0_per_thread<D>(); ++i) {
    const int e = threadIdx.x + i * kBlock, b = e / HALF, r = e % HALF;
    const int fl = r / (D / 2), a = 2 * (r % (D / 2));
    buf[i] = *reinterpret_cast<const float4 *>(src + fb[fl] + (uint32_t)a + (uint32_t)b * sj);
  }
}

template <int D>
__device__ __forceinline__ void m0_lds_put(float2 *tile, const float4 (&buf)[m0_per_thread<D>()]) {
  constexpr int HALF = lds_fibers<D>() * D / 2, ST = D * D + 1;
#pragma unroll
  for (int i = 0; i < m0_per_thread<D>(); ++i) {
    const int e = threadIdx.x + i * kBlock, b = e / HALF, r = e % HALF;
    const int fl = r / (D / 2), a = 2 * (r % (D / 2));
    float2 *tp = tile + fl * ST + b * D + a;
    tp[0] = make_float2(buf[i].x, buf[i].y);
    tp[1] = make_float2(buf[i].z, buf[i].w);
  }
}

template <int D>
__device__ __forceinline__ void m0_gstore(float2 *dst, const uint32_t *fb, uint32_t sj, const float2 *tile) {
  constexpr int HALF = lds_fibers<D>() * D / 2, ST = D * D + 1;
#pragma unroll
  for (int i = 0; i < m0_per_thread<D>(); ++i) {
    const int e = threadIdx.x + i * kBlock, b = e / HALF, r = e % HALF;
    const int fl = r / (D / 2), a = 2 * (r % (D / 2));
    const float2 *tp = tile + fl * ST + b * D + a;
    *reinterpret_cast<float4 *>(dst + fb[fl] + (uint32_t)a + (uint32_t)b * sj) =
        make_float4(tp[0].x, tp[0].y, tp[1].x, tp[1].y);
  }
}

// tile: m0_tile_elems<D>() float2, fbase: 2 x lds_fibers<D>() words of LDS.
// Contains barriers: every thread of the workgroup must call it.
template <int D, int KIND, bool DAG>
__device__ __forceinline__ void gate2_m0p_block(int vb, const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                                const GateLaunch &g, float2 *tile, uint32_t (*fbase)[lds_fibers<D>()]) {
  constexpr int ST = D * D + 1;
  const uint32_t t0 = (uint32_t)vb * kM0Tiles;
  float4 buf[m0_per_thread<D>()];
  m0_bases<D>(t0, g, fbase[0]);
  if (kM0Tiles > 1) m0_bases<D>(t0 + 1, g, fbase[1]);
  __syncthreads();
  m0_gload<D>(src, fbase[0], g.sj, buf);
  m0_lds_put<D>(tile, buf);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll 1
  for (int t = 0; t < kM0Tiles; ++t) {
    const bool more = t + 1 < kM0Tiles;
    if (more) m0_gload<D>(src, fbase[(t + 1) & 1], g.sj, buf);
    float2 *base = tile + lane * ST;
    switch (wave) {
      case 0: gate_group<D, KIND, DAG, 4, 0>(base, base, 1u, (uint32_t)D, U); break;
      case 1: gate_group<D, KIND, DAG, 4, 1>(base, base, 1u, (uint32_t)D, U); break;
      case 2: gate_group<D, KIND, DAG, 4, 2>(base, base, 1u, (uint32_t)D, U); break;
      default: gate_group<D, KIND, DAG, 4, 3>(base, base, 1u, (uint32_t)D, U); break;
    }
    __syncthreads();
    m0_gstore<D>(psi, fbase[t & 1], g.sj, tile);
    __syncthreads();
    if (more) {
      m0_lds_put<D>(tile, buf);
      if (t + 2 < kM0Tiles) m0_bases<D>(t0 + t + 2, g, fbase[t & 1]);
      __syncthreads();
    }
  }
}

template <int D, int KIND, bool DAG>
__global__ __launch_bounds__(kBlock) void k_gate2_m0p(const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                                      GateLaunch g) {
  __shared__ float2 tile[m0_tile_elems<D>()];
  __shared__ uint32_t fbase[2][lds_fibers<D>()];
  gate2_m0p_block<D, KIND, DAG>(xcd_remap(blockIdx.x, gridDim.x), src, psi, U, g, tile, fbase);
}

// Reverse step over the workgroup's kM0Tiles tiles; returns the thread's sum of
// Re<lam|A phi> over all of them.  tp, tl: m0_tile_elems<D>() float2 each,
// fbase: 2 x lds_fibers<D>() words of LDS.  Contains barriers.
template <int D, int KIND, bool WPHI = true>
__device__ __forceinline__ float adj_m0p_block(int vb, float2 *phi, float2 *lam, const float2 *__restrict__ U,
                                               const float2 *__restrict__ A, const GateLaunch &g, float2 *tp,
                                               float2 *tl, uint32_t (*fbase)[lds_fibers<D>()]) {
  constexpr int ST = D * D + 1;
  const uint32_t t0 = (uint32_t)vb * kM0Tiles;
  float4 bp[m0_per_thread<D>()], bl[m0_per_thread<D>()];
  m0_bases<D>(t0, g, fbase[0]);
  if (kM0Tiles > 1) m0_bases<D>(t0 + 1, g, fbase[1]);
  __syncthreads();
  m0_gload<D>(phi, fbase[0], g.sj, bp);
  m0_gload<D>(lam, fbase[0], g.sj, bl);
  m0_lds_put<D>(tp, bp);
  m0_lds_put<D>(tl, bl);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float gacc = 0.f;
#pragma unroll 1
  for (int t = 0; t < kM0Tiles; ++t) {
    const bool more = t + 1 < kM0Tiles;
    if (more) {
      m0_gload<D>(phi, fbase[(t + 1) & 1], g.sj, bp);
      m0_gload<D>(lam, fbase[(t + 1) & 1], g.sj, bl);
    }
    float2 *pb = tp + lane * ST, *lb = tl + lane * ST;
    switch (wave) {
      case 0: gacc += adj_group<D, KIND, 4, 0, WPHI>(pb, lb, 1u, (uint32_t)D, U, A); break;
      case 1: gacc += adj_group<D, KIND, 4, 1, WPHI>(pb, lb, 1u, (uint32_t)D, U, A); break;
      case 2: gacc += adj_group<D, KIND, 4, 2, WPHI>(pb, lb, 1u, (uint32_t)D, U, A); break;
      default: gacc += adj_group<D, KIND, 4, 3, WPHI>(pb, lb, 1u, (uint32_t)D, U, A); break;
    }
    __syncthreads();
    if (WPHI) m0_gstore<D>(phi, fbase[t & 1], g.sj, tp);
    m0_gstore<D>(lam, fbase[t & 1], g.sj, tl);
    __syncthreads();
    if (more) {
      m0_lds_put<D>(tp, bp);
      m0_lds_put<D>(tl, bl);
      if (t + 2 < kM0Tiles) m0_bases<D>(t0 + t + 2, g, fbase[t & 1]);
      __syncthreads();
    }
  }
  return gacc;
}

template <int D, int KIND, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_gate2_adj_m0p(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                          const float2 *__restrict__ U, const float2 *__restrict__ A,
                                                          double *__restrict__ partial, GateLaunch g) {
  __shared__ float2 tp[m0_tile_elems<D>()], tl[m0_tile_elems<D>()];
  __shared__ uint32_t fbase[2][lds_fibers<D>()];
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const float gacc = adj_m0p_block<D, KIND, WPHI>(vb, phi, lam, U, A, g, tp, tl, fbase);
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

template <int D, int KIND, bool DAG>
__global__ __launch_bounds__(kBlock) void k_gate2_m0(const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                                     GateLaunch g) {
  __shared__ float2 tile[m0_tile_elems<D>()];
  __shared__ uint32_t fbase[lds_fibers<D>()];
  gate2_m0_block<D, KIND, DAG>(xcd_remap(blockIdx.x, gridDim.x), src, psi, U, g, tile, fbase);
}

template <int D, int KIND, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_gate2_adj_m0(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                         const float2 *__restrict__ U, const float2 *__restrict__ A,
                                                         double *__restrict__ partial, GateLaunch g) {
  __shared__ float2 tp[m0_tile_elems<D>()], tl[m0_tile_elems<D>()];
  __shared__ uint32_t fbase[lds_fibers<D>()];
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const float gacc = adj_m0_block<D, KIND, WPHI>(vb, phi, lam, U, A, g, tp, tl, fbase);
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

// ---------------------------------------------------------------- single-mode diagonal gates
// O = exp(theta A) with A = i f(N_r) is diag(exp(i theta f(n_r))); f = n^2 (KERR) or n (ROT).
struct DiagLaunch {
  int nrows, r, kerr;
  FastDiv dsr;  // divide a row index by d^(r-1) (r >= 1)
};

// phs: kMaxD float2 of LDS.  Contains a barrier.
template <int D, bool DAG>
__device__ __forceinline__ void diag_block(int vb, const float2 *src, float2 *psi, const float2 *__restrict__ phg,
                                           const DiagLaunch &a, float2 *phs) {
  if (threadIdx.x < D) {
    const float2 p = phg[threadIdx.x];
    phs[threadIdx.x] = DAG ? make_float2(p.x, -p.y) : p;
  }
  __syncthreads();
  const int row = vb * kBlock + threadIdx.x;
  if (row < a.nrows) {
    float2 v[D];
    load_row<D>(src + (size_t)row * D, v);
    const int n = a.r == 0 ? 0 : (int)(fdiv((uint32_t)row, a.dsr) % D);
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const float2 p = phs[a.r == 0 ? q : n];
      float2 o = make_float2(0.f, 0.f);
      cmac(o, p, v[q]);
      v[q] = o;
    }
    store_row<D>(psi + (size_t)row * D, v);
  }
  __syncthreads();
}

template <int D, bool WPHI = true>
__device__ __forceinline__ float diag_adj_block(int vb, float2 *phi, float2 *lam, const float2 *__restrict__ phg,
                                                const DiagLaunch &a, float2 *phs) {
  if (threadIdx.x < D) phs[threadIdx.x] = phg[threadIdx.x];
  __syncthreads();
  const int row = vb * kBlock + threadIdx.x;
  float gacc = 0.f;
  if (row < a.nrows) {
    float2 pv[D], lv[D];
    load_row<D>(phi + (size_t)row * D, pv);
    load_row<D>(lam + (size_t)row * D, lv);
    const int n = a.r == 0 ? 0 : (int)(fdiv((uint32_t)row, a.dsr) % D);
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const int lev = a.r == 0 ? q : n;
      const float f = a.kerr ? (float)(lev * lev) : (float)lev;
      // Re(conj(lam) * i f phi) = -f Im(conj(lam) phi)
      gacc = fmaf(-f, lv[q].x * pv[q].y - lv[q].y * pv[q].x, gacc);
      const float2 p = phs[lev];
      float2 np = make_float2(0.f, 0.f), nl = make_float2(0.f, 0.f);
      if (WPHI) cmac_conj(np, p, pv[q]);
      cmac_conj(nl, p, lv[q]);
      pv[q] = np;
      lv[q] = nl;
    }
    if (WPHI) store_row<D>(phi + (size_t)row * D, pv);
    store_row<D>(lam + (size_t)row * D, lv);
  }
  __syncthreads();
  return gacc;
}

template <int D, bool DAG>
__global__ __launch_bounds__(kBlock) void k_diag(const float2 *src, float2 *psi, const float2 *__restrict__ phg,
                                                 DiagLaunch a) {
  __shared__ float2 phs[kMaxD];
  diag_block<D, DAG>(xcd_remap(blockIdx.x, gridDim.x), src, psi, phg, a, phs);
}

template <int D, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_diag_adj(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                     const float2 *__restrict__ phg, double *__restrict__ partial,
                                                     DiagLaunch a) {
  __shared__ float2 phs[kMaxD];
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const float gacc = diag_adj_block<D, WPHI>(vb, phi, lam, phg, a, phs);
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

// ---------------------------------------------------------------- runs of single-mode phase gates
// Consecutive gates exp(theta_g i f_g(N_{r_g})) (f = n^2 or n) commute and
// multiply into one diagonal unitary: amplitude n picks up the product of the
// gates' phase-table entries at n_{r_g}.  One pass applies a whole run.  In the
// reverse sweep every gate of the run sees the same Im(conj(lam) phi) per
// amplitude (a diagonal phase leaves conj(lam) phi unchanged), so one pass also
// yields all of the run's gradient partials: per row, M_k = sum_q q^k m_q with
// m_q = Im(conj(lam) phi) at n_0 = q; a gate on mode 0 takes -M_2 (Kerr) or -M_1
// (rotation), a gate on mode r >= 1 takes -f(n_r) M_0.
// Stage the run's phase tables (conjugated when DAG) in LDS: tb[g * D + n] for
// the gates on modes r >= 1 and t0[q] = product over the mode-0 gates.
template <int D, bool DAG>
__device__ __forceinline__ void diag_run_tables(const float2 *__restrict__ U, const DiagRun &a, float2 *tb,
                                                float2 *t0) {
  for (int e = threadIdx.x; e < a.ng * D; e += kBlock) {
    const float2 v = U[(size_t)(e / D) * a.stride + e % D];
    tb[e] = DAG ? make_float2(v.x, -v.y) : v;
  }
  __syncthreads();
  if (threadIdx.x < D) {
    float2 p = make_float2(1.f, 0.f);
    for (int g = 0; g < a.ng; ++g)
      if (a.r[g] == 0) {
        const float2 t = tb[g * D + threadIdx.x];
        p = make_float2(p.x * t.x - p.y * t.y, p.x * t.y + p.y * t.x);
      }
    t0[threadIdx.x] = p;
  }
  __syncthreads();
}

// Product of the row's phases from the gates on modes r >= 1.
template <int D>
__device__ __forceinline__ float2 diag_run_row_phase(int row, const DiagRun &a, const float2 *tb) {
  float2 p = make_float2(1.f, 0.f);
  for (int g = 0; g < a.ng; ++g)
    if (a.r[g] > 0) {
      const int n = (int)(fdiv((uint32_t)row, a.dsr[g]) % D);
      const float2 t = tb[g * D + n];
      p = make_float2(p.x * t.x - p.y * t.y, p.x * t.y + p.y * t.x);
    }
  return p;
}

// tb: kMaxDiagRun * kMaxD, t0: kMaxD float2 of LDS.  Contains barriers.
template <int D, bool DAG>
__device__ __forceinline__ void diag_run_block(int vb, const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                               const DiagRun &a, float2 *tb, float2 *t0) {
  diag_run_tables<D, DAG>(U, a, tb, t0);
  const int row = vb * kBlock + threadIdx.x;
  if (row < a.nrows) {
    float2 v[D];
    load_row<D>(src + (size_t)row * D, v);
    const float2 pr = diag_run_row_phase<D>(row, a, tb);
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const float2 t = t0[q];
      const float2 ph = make_float2(pr.x * t.x - pr.y * t.y, pr.x * t.y + pr.y * t.x);
      float2 o = make_float2(0.f, 0.f);
      cmac(o, ph, v[q]);
      v[q] = o;
    }
    store_row<D>(psi + (size_t)row * D, v);
  }
  __syncthreads();
}

// Reverse step of a run: red[w][g] (LDS, 4 x kMaxDiagRun doubles) receives the
// wavefront sums of each gate's Re<lam|A_g phi>; phi (when WPHI) and lam are
// multiplied by the conjugate phase.  Contains barriers.
template <int D, bool WPHI>
__device__ __forceinline__ void diag_run_adj_block(int vb, float2 *phi, float2 *lam, const float2 *__restrict__ U,
                                                   const DiagRun &a, float2 *tb, float2 *t0,
                                                   double (*red)[kMaxDiagRun]) {
  diag_run_tables<D, true>(U, a, tb, t0);
  const int row = vb * kBlock + threadIdx.x;
  float m0 = 0.f, m1 = 0.f, m2 = 0.f;
  if (row < a.nrows) {
    float2 pv[D], lv[D];
    load_row<D>(phi + (size_t)row * D, pv);
    load_row<D>(lam + (size_t)row * D, lv);
    const float2 pr = diag_run_row_phase<D>(row, a, tb);
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const float m = lv[q].x * pv[q].y - lv[q].y * pv[q].x;
      m0 += m;
      m1 += (float)q * m;
      m2 += (float)(q * q) * m;
      const float2 t = t0[q];
      const float2 ph = make_float2(pr.x * t.x - pr.y * t.y, pr.x * t.y + pr.y * t.x);
      float2 np = make_float2(0.f, 0.f), nl = make_float2(0.f, 0.f);
      if (WPHI) cmac(np, ph, pv[q]);
      cmac(nl, ph, lv[q]);
      pv[q] = np;
      lv[q] = nl;
    }
    if (WPHI) store_row<D>(phi + (size_t)row * D, pv);
    store_row<D>(lam + (size_t)row * D, lv);
  }
  const bool in = row < a.nrows;
  for (int g = 0; g < a.ng; ++g) {
    float v;
    if (a.r[g] == 0) {
      v = a.kerr[g] ? -m2 : -m1;
    } else {
      const int n = in ? (int)(fdiv((uint32_t)row, a.dsr[g]) % D) : 0;
      v = -(a.kerr[g] ? (float)(n * n) : (float)n) * m0;
    }
    const double sv = wave_sum_d(in ? (double)v : 0.0);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][g] = sv;
  }
  __syncthreads();
}

template <int D, bool DAG>
__global__ __launch_bounds__(kBlock) void k_diag_run(const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                                     DiagRun a) {
  __shared__ float2 tb[kMaxDiagRun * kMaxD], t0[kMaxD];
  diag_run_block<D, DAG>(xcd_remap(blockIdx.x, gridDim.x), src, psi, U, a, tb, t0);
}

// partial[g * rs + vb]: gate g's sum over workgroup vb.
template <int D, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_diag_run_adj(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                         const float2 *__restrict__ U, double *__restrict__ partial,
                                                         int rs, DiagRun a) {
  __shared__ float2 tb[kMaxDiagRun * kMaxD], t0[kMaxD];
  __shared__ double red[kBlock / 64][kMaxDiagRun];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  diag_run_adj_block<D, WPHI>(vb, phi, lam, U, a, tb, t0, red);
  if ((int)threadIdx.x < a.ng) {
    const int g = threadIdx.x;
    partial[(size_t)g * rs + vb] = (red[0][g] + red[1][g]) + (red[2][g] + red[3][g]);
  }
}

template <int D>
constexpr int lds_fibers_d() { return lds_fibers<D>(); }

template <int D>
int fibers_per_block_d(int i) { return i == 0 ? lds_fibers<D>() : 64 * (4 / direct_groups<D>()); }

// The pipelined mode-0 kernels: d = 8 and whole tiles for every workgroup.
template <int D>
constexpr bool m0p_used(int i, uint32_t nfib) {
  return D == 8 && i == 0 && nfib % (uint32_t)(lds_fibers<D>() * kM0Tiles) == 0;
}

// Fibres per workgroup of the kernels gate_launch_d / adj_launch_d launch.
template <int D>
int launch_fibers_per_block_d(int i, uint32_t nfib) {
  return m0p_used<D>(i, nfib) ? lds_fibers<D>() * kM0Tiles : fibers_per_block_d<D>(i);
}

template <int D>
void gate_launch_d(const GateLaunch &gl, int i, int kind, bool dag, const float2 *U, const float2 *src, float2 *psi,
                   int G, hipStream_t s) {
#define GATE_K(KN, K, DG) hipLaunchKernelGGL((KN<D, K, DG>), dim3(G), dim3(kBlock), 0, s, src, psi, U, gl)
#define GATE_SEL(KN)                                                         \
  if (kind == KIND_SUM) {                                                    \
    if (dag) GATE_K(KN, KIND_SUM, true); else GATE_K(KN, KIND_SUM, false);   \
  } else {                                                                   \
    if (dag) GATE_K(KN, KIND_DIFF, true); else GATE_K(KN, KIND_DIFF, false); \
  }
  if (i == 0) {
    bool piped = false;
    if constexpr (D == 8) {
      if (m0p_used<D>(i, gl.nfib)) {
        GATE_SEL(k_gate2_m0p);
        piped = true;
      }
    }
    if (!piped) GATE_SEL(k_gate2_m0);
  } else {
    GATE_SEL(k_gate2);
  }
#undef GATE_SEL
#undef GATE_K
}

template <int D>
void adj_launch_d(const GateLaunch &gl, int i, int kind, const float2 *U, const float2 *A, float2 *phi, float2 *lam,
                  double *partial, int G, bool wphi, hipStream_t s) {
#define ADJ_K(KN, K, W) hipLaunchKernelGGL((KN<D, K, W>), dim3(G), dim3(kBlock), 0, s, phi, lam, U, A, partial, gl)
#define ADJ_SEL(KN)                                                      \
  if (kind == KIND_SUM) {                                                \
    if (wphi) ADJ_K(KN, KIND_SUM, true); else ADJ_K(KN, KIND_SUM, false);    \
  } else {                                                               \
    if (wphi) ADJ_K(KN, KIND_DIFF, true); else ADJ_K(KN, KIND_DIFF, false);  \
  }
  if (i == 0) {
    bool piped = false;
    if constexpr (D == 8) {
      if (m0p_used<D>(i, gl.nfib)) {
        ADJ_SEL(k_gate2_adj_m0p);
        piped = true;
      }
    }
    if (!piped) ADJ_SEL(k_gate2_adj_m0);
  } else {
    ADJ_SEL(k_gate2_adj);
  }
#undef ADJ_SEL
#undef ADJ_K
}

#define FOCK_GATE_INSTANTIATE(D)                                                                             \
  template int fibers_per_block_d<D>(int);                                                                 \
  template int launch_fibers_per_block_d<D>(int, uint32_t);                                                \
  template void gate_launch_d<D>(const GateLaunch &, int, int, bool, const float2 *, const float2 *,       \
                                 float2 *, int, hipStream_t);                                              \
  template void adj_launch_d<D>(const GateLaunch &, int, int, const float2 *, const float2 *, float2 *,    \
                                float2 *, double *, int, bool, hipStream_t);
#define FOCK_GATE_EXTERN(D)                                                                                  \
  extern template int fibers_per_block_d<D>(int);                                                          \
  extern template int launch_fibers_per_block_d<D>(int, uint32_t);                                         \
  extern template void gate_launch_d<D>(const GateLaunch &, int, int, bool, const float2 *, const float2 *, \
                                        float2 *, int, hipStream_t);                                       \
  extern template void adj_launch_d<D>(const GateLaunch &, int, int, const float2 *, const float2 *,       \
                                       float2 *, float2 *, double *, int, bool, hipStream_t);

}  // namespace fock
