// Hamiltonian stencil H psi with fused FP64 energy/norm partials, and the
// fixed-order FP64 reduction.
//
// H (Sec. III, build sign convention):
//   H = sum_bonds [ -J (a_i^+ a_j + h.c.) + Delta (a_i a_j + h.c.) ]
//     + sum_r [ (U/2 + K) n_r (n_r - 1) - mu n_r ]
// Matrix elements from the truncated ladder action (Sec. II.A):
//   (a_i^+ a_j psi)[n] = sqrt(n_i) sqrt(n_j + 1) psi[n - e_i + e_j]   (0 if n_j = d-1)
//   (a_i a_j psi)[n]   = sqrt(n_i + 1) sqrt(n_j + 1) psi[n + e_i + e_j]
//   (a_i^+ a_j^+ psi)[n] = sqrt(n_i) sqrt(n_j) psi[n - e_i - e_j]
//
// Work decomposition: one thread per "row", i.e. the d consecutive amplitudes
// along mode 0 (stride 1) for fixed n_1..n_{L-1}.  A bond (r, r+1) with r >= 1
// has row-uniform coefficients, so each of its four neighbour terms is one
// coalesced row load plus 2d FMAs.  Bonds touching mode 0 read the rows
// n_j +- 1 and shift them by one position along the row.
#include "device_common.h"

namespace fock {

// LDS tile: the rows whose digits n_1..n_K take all values for fixed higher
// digits, i.e. D^(K+1) consecutive amplitudes.  Bonds among modes 0..K read
// their neighbours from LDS; bonds reaching mode K+1 or beyond read rows from
// global memory (L2).  The row stride in LDS is padded so that the 16-byte
// row loads of consecutive threads fall in different bank groups.
template <int D>
struct TileCfg {
  static constexpr int RS = (D % 2 == 0) ? D + 2 : D + 1;  // LDS row stride (float2)
  static constexpr int MAXROWS = (4096 / D) < 512 ? (4096 / D) : 512;
};

__device__ __forceinline__ int tile_k(int L, int D, int maxrows) {
  int k = 0, t = 1;
  while (k < L - 1 && t * D <= maxrows) {
    t *= D;
    ++k;
  }
  return k;
}

template <int D>
__device__ __forceinline__ void lds_row(const float2 *tile, int r, float2 (&v)[D]) {
  constexpr int RS = TileCfg<D>::RS;
  if constexpr (D % 2 == 0) {
    const float4 *q = reinterpret_cast<const float4 *>(tile + r * RS);
#pragma unroll
    for (int k = 0; k < D / 2; ++k) {
      const float4 t = q[k];
      v[2 * k] = make_float2(t.x, t.y);
      v[2 * k + 1] = make_float2(t.z, t.w);
    }
  } else {
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = tile[r * RS + k];
  }
}

template <int D>
__device__ __forceinline__ void axpy_v(float2 (&acc)[D], const float2 (&v)[D], float c) {
#pragma unroll
  for (int q = 0; q < D; ++q) {
    acc[q].x = fmaf(c, v[q].x, acc[q].x);
    acc[q].y = fmaf(c, v[q].y, acc[q].y);
  }
}

// Copy T rows (T * D amplitudes starting at row r0) into the padded tile.
template <int D>
__device__ __forceinline__ void load_tile(float2 *tile, const float2 *__restrict__ psi, int r0, int T) {
  constexpr int RS = TileCfg<D>::RS;
  const float2 *src = psi + (size_t)r0 * D;
  if constexpr (D % 2 == 0) {
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    for (int e = threadIdx.x; e < T * D / 2; e += kBlock) {
      const int r = e / (D / 2), c = e % (D / 2);
      reinterpret_cast<float4 *>(tile + r * RS)[c] = s4[e];
    }
  } else {
    for (int e = threadIdx.x; e < T * D; e += kBlock) tile[(e / D) * RS + e % D] = src[e];
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_apply_h(const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                                    double *__restrict__ partial, HamArgs h) {
  __shared__ double red[4];
  __shared__ float4 tile4[(TileCfg<D>::MAXROWS * TileCfg<D>::RS + 1) / 2];
  float2 *tile = reinterpret_cast<float2 *>(tile4);
  const int K = tile_k(h.L, D, TileCfg<D>::MAXROWS);
  int T = 1;
  for (int k = 0; k < K; ++k) T *= D;
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const int r0 = vb * T;
  load_tile<D>(tile, psi, r0, T);
  __syncthreads();
  const float J = h.J, Dl = h.Delta;
  float e = 0.f, nn = 0.f;
  for (int lr = threadIdx.x; lr < T; lr += kBlock) {
    const int row = r0 + lr;
    float2 acc[D], own[D];
#pragma unroll
    for (int q = 0; q < D; ++q) acc[q] = make_float2(0.f, 0.f);
    lds_row<D>(tile, lr, own);
    // digits of this row (4 bits per mode) and the diagonal part of modes >= 1
    float dg_row = 0.f;
    uint64_t dlo = 0, dhi = 0;
    {
      uint32_t t = (uint32_t)row;
      for (int r = 1; r < h.L; ++r) {
        const uint32_t n = t % D;
        t /= D;
        const float nf = (float)n;
        dg_row += h.c2 * nf * (nf - 1.f) - h.mu * nf;
        if (r < 16) dlo |= (uint64_t)n << (4 * r);
        else dhi |= (uint64_t)n << (4 * (r - 16));
      }
    }
    auto digit = [&](int r) -> int {
      return (int)((r < 16 ? (dlo >> (4 * r)) : (dhi >> (4 * (r - 16)))) & 15ull);
    };
    const int n1 = h.L >= 2 ? digit(1) : 0;
    const int nprev = digit(h.L - 1);
    // bonds (r-1, r) inside the tile: neighbours from LDS
    const int rin = K < h.L - 1 ? K : h.L - 1;
    for (int r = 2; r <= rin; ++r) {
      const int ni = digit(r - 1), nj = digit(r);
      const int si = h.srow[r - 1], sj = h.srow[r];
      const float smi = sqrtf((float)ni), spi = sqrtf((float)ni + 1.f);
      const float smj = sqrtf((float)nj), spj = sqrtf((float)nj + 1.f);
      float2 v[D];
      if (J != 0.f) {
        if (ni >= 1 && nj <= D - 2) { lds_row<D>(tile, lr - si + sj, v); axpy_v<D>(acc, v, -J * smi * spj); }
        if (ni <= D - 2 && nj >= 1) { lds_row<D>(tile, lr + si - sj, v); axpy_v<D>(acc, v, -J * spi * smj); }
      }
      if (Dl != 0.f) {
        if (ni <= D - 2 && nj <= D - 2) { lds_row<D>(tile, lr + si + sj, v); axpy_v<D>(acc, v, Dl * spi * spj); }
        if (ni >= 1 && nj >= 1) { lds_row<D>(tile, lr - si - sj, v); axpy_v<D>(acc, v, Dl * smi * smj); }
      }
    }
    // bonds reaching beyond the tile: all neighbour rows of a bond are loaded
    // unconditionally (an invalid neighbour reads the row itself with weight
    // 0) so that the loads of a bond, and of two bonds per iteration, are in
    // flight together.
    {
      int r = (K + 1 > 2) ? K + 1 : 2;
      auto bond_offsets = [&](int rr, int (&off)[4], float (&cf)[4]) {
        const int ni = digit(rr - 1), nj = digit(rr);
        const int si = h.srow[rr - 1], sj = h.srow[rr];
        const float smi = sqrtf((float)ni), spi = sqrtf((float)ni + 1.f);
        const float smj = sqrtf((float)nj), spj = sqrtf((float)nj + 1.f);
        const bool v0 = ni >= 1 && nj <= D - 2, v1 = ni <= D - 2 && nj >= 1;
        const bool v2 = ni <= D - 2 && nj <= D - 2, v3 = ni >= 1 && nj >= 1;
        off[0] = v0 ? -si + sj : 0; cf[0] = v0 ? -J * smi * spj : 0.f;
        off[1] = v1 ? si - sj : 0;  cf[1] = v1 ? -J * spi * smj : 0.f;
        off[2] = v2 ? si + sj : 0;  cf[2] = v2 ? Dl * spi * spj : 0.f;
        off[3] = v3 ? -si - sj : 0; cf[3] = v3 ? Dl * smi * smj : 0.f;
      };
      const int nt = Dl != 0.f ? 4 : 2;  // pairing terms only when Delta != 0
      for (; r + 1 < h.L; r += 2) {
        int oa[4], ob[4];
        float ca[4], cb[4];
        bond_offsets(r, oa, ca);
        bond_offsets(r + 1, ob, cb);
        float2 va[4][D], vb2[4][D];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < nt) {
            load_row<D>(psi + (size_t)(row + oa[k]) * D, va[k]);
            load_row<D>(psi + (size_t)(row + ob[k]) * D, vb2[k]);
          }
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < nt) {
            axpy_v<D>(acc, va[k], ca[k]);
            axpy_v<D>(acc, vb2[k], cb[k]);
          }
      }
      if (r < h.L) {
        int oa[4];
        float ca[4];
        bond_offsets(r, oa, ca);
        float2 va[4][D];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < nt) load_row<D>(psi + (size_t)(row + oa[k]) * D, va[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < nt) axpy_v<D>(acc, va[k], ca[k]);
      }
    }
    // bonds touching mode 0: (0, 1) and the ring bond (0, L-1)
    const int nb0 = (h.L >= 2 ? 1 : 0) + h.periodic_wrap;
    for (int b = 0; b < nb0; ++b) {
      const int j = (b == 0) ? 1 : h.L - 1;
      const int nj = (b == 0) ? n1 : nprev;
      const int sj = h.srow[j];
      const bool in_tile = j <= K;
      if (nj <= D - 2) {
        float2 P[D];
        if (in_tile) lds_row<D>(tile, lr + sj, P);
        else load_row<D>(psi + (size_t)(row + sj) * D, P);
        const float spj = sqrtf((float)nj + 1.f);
        if (J != 0.f) {
          const float c = -J * spj;  // a_0^+ a_j : out[q] <- sqrt(q) P[q-1]
#pragma unroll
          for (int q = 1; q < D; ++q) {
            acc[q].x = fmaf(c * h.sq[q], P[q - 1].x, acc[q].x);
            acc[q].y = fmaf(c * h.sq[q], P[q - 1].y, acc[q].y);
          }
        }
        if (Dl != 0.f) {
          const float c = Dl * spj;  // a_0 a_j : out[q] <- sqrt(q+1) P[q+1]
#pragma unroll
          for (int q = 0; q < D - 1; ++q) {
            acc[q].x = fmaf(c * h.sq[q + 1], P[q + 1].x, acc[q].x);
            acc[q].y = fmaf(c * h.sq[q + 1], P[q + 1].y, acc[q].y);
          }
        }
      }
      if (nj >= 1) {
        float2 M[D];
        if (in_tile) lds_row<D>(tile, lr - sj, M);
        else load_row<D>(psi + (size_t)(row - sj) * D, M);
        const float smj = sqrtf((float)nj);
        if (J != 0.f) {
          const float c = -J * smj;  // a_j^+ a_0 : out[q] <- sqrt(q+1) M[q+1]
#pragma unroll
          for (int q = 0; q < D - 1; ++q) {
            acc[q].x = fmaf(c * h.sq[q + 1], M[q + 1].x, acc[q].x);
            acc[q].y = fmaf(c * h.sq[q + 1], M[q + 1].y, acc[q].y);
          }
        }
        if (Dl != 0.f) {
          const float c = Dl * smj;  // a_0^+ a_j^+ : out[q] <- sqrt(q) M[q-1]
#pragma unroll
          for (int q = 1; q < D; ++q) {
            acc[q].x = fmaf(c * h.sq[q], M[q - 1].x, acc[q].x);
            acc[q].y = fmaf(c * h.sq[q], M[q - 1].y, acc[q].y);
          }
        }
      }
    }
    // diagonal, energy and norm
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const float qf = (float)q;
      const float dg = dg_row + h.c2 * qf * (qf - 1.f) - h.mu * qf;
      acc[q].x = fmaf(dg, own[q].x, acc[q].x);
      acc[q].y = fmaf(dg, own[q].y, acc[q].y);
      e = fmaf(own[q].x, acc[q].x, fmaf(own[q].y, acc[q].y, e));
      nn = fmaf(own[q].x, own[q].x, fmaf(own[q].y, own[q].y, nn));
    }
    store_row<D>(hpsi + (size_t)row * D, acc);
  }
  const double se = block_sum_d((double)e, red);
  const double sn = block_sum_d((double)nn, red);
  if (threadIdx.x == 0) {
    partial[2 * vb] = se;
    partial[2 * vb + 1] = sn;
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double *__restrict__ partial, int nblocks, int ncols,
                                                   double *__restrict__ out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partial[(size_t)b * ncols + c];
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) out[c] = s;
}

__global__ __launch_bounds__(kBlock) void k_reduce_rows(const double *__restrict__ partial, int row_stride,
                                                        const GateRec *__restrict__ recs, double *__restrict__ out) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  const int nb = recs[k].nblk;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) s += partial[(size_t)k * row_stride + b];
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) out[k] = s;
}

int launch_reduce_rows(const double *partial, int row_stride, const GateRec *recs, int n, double *out,
                       hipStream_t s) {
  if (n <= 0) return FOCK_OK;
  hipLaunchKernelGGL(k_reduce_rows, dim3(n), dim3(kBlock), 0, s, partial, row_stride, recs, out);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

// Rows per workgroup tile (D^K, see TileCfg / tile_k).
template <int D>
static int tile_rows_d(int L) {
  int k = 0, t = 1;
  while (k < L - 1 && t * D <= TileCfg<D>::MAXROWS) {
    t *= D;
    ++k;
  }
  return t;
}

int apply_h_tile_rows(int L, int d) {
  switch (d) {
#define CASE(D) \
  case D: return tile_rows_d<D>(L);
    CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13)
    CASE(14) CASE(15) CASE(16)
#undef CASE
    default: return 1;
  }
}

int apply_h_blocks(const HamArgs &h) { return h.nrows / apply_h_tile_rows(h.L, h.d); }

template <int D>
static void launch_h_t(const HamArgs &h, const float2 *psi, float2 *hpsi, double *partial, int G, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_h<D>, dim3(G), dim3(kBlock), 0, s, psi, hpsi, partial, h);
}

int launch_apply_h(const HamArgs &h, const float2 *psi, float2 *hpsi, double *partial, int *nblocks,
                   hipStream_t s) {
  const int G = apply_h_blocks(h);
  *nblocks = G;
  switch (h.d) {
#define CASE(D) \
  case D: launch_h_t<D>(h, psi, hpsi, partial, G, s); break;
    CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13)
    CASE(14) CASE(15) CASE(16)
#undef CASE
    default: return set_error(FOCK_ERR_UNSUPPORTED, "d=%d unsupported", h.d);
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_reduce(const double *partial, int nblocks, int ncols, double *out, hipStream_t s) {
  if (ncols <= 0) return FOCK_OK;
  hipLaunchKernelGGL(k_reduce, dim3(ncols), dim3(kBlock), 0, s, partial, nblocks, ncols, out);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
