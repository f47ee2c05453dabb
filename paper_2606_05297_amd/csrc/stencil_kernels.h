// Device functions of the stencil-type kernels (H psi and pool scoring),
// shared by the single-point kernels and the batched sweep kernels.
#pragma once

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
  static constexpr int PWORDS = (MAXROWS * RS + 1) / 2;     // float4 words of a tile
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

// Work of tile vb: H psi on its rows; e, nn receive this thread's share of
// <psi|H|psi> and <psi|psi>.  tile: TileCfg<D>::PWORDS float4 of LDS
// (16-byte aligned).  Contains barriers: every thread must call it.
template <int D>
__device__ __forceinline__ void hblock(int vb, const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                       const HamArgs &h, float2 *tile, float &e_out, float &nn_out) {
  const int K = tile_k(h.L, D, TileCfg<D>::MAXROWS);
  int T = 1;
  for (int k = 0; k < K; ++k) T *= D;
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
      const int rend = h.L - h.hi_m + (h.hi_m > 0 ? 1 : 0);  // bonds (r-1, r) with r < rend are this pass's
      for (; r + 1 < rend; r += 2) {
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
      if (r < rend) {
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
    const int nb0 = (h.L >= 2 ? 1 : 0) + (h.hi_m > 0 ? 0 : h.periodic_wrap);
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
    // two-pass: the first pass left its bonds' share of this row in hpsi
    if (h.hi_m > 0) {
      float2 pa[D];
      load_row<D>(hpsi + (size_t)row * D, pa);
#pragma unroll
      for (int q = 0; q < D; ++q) {
        acc[q].x += pa[q].x;
        acc[q].y += pa[q].y;
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
  e_out = e;
  nn_out = nn;
  __syncthreads();
}


// First pass of the two-pass stencil.  Tile t holds the rows whose digits of
// the top m = h.hi_m modes take all values, for fixed digits of modes
// 1..L-1-m (row = t + lr S, S = d^(L-1-m), lr = the top digits).  It applies
// the bonds among the top modes and the ring bond (0, L-1) with neighbours
// from LDS and writes that share of H psi; the second pass (hblock with
// hi_m > 0) adds the remaining bonds and the diagonal in place.
template <int D>
__device__ __forceinline__ void hblock_hi(int t, const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                          const HamArgs &h, float2 *tile) {
  constexpr int RS = TileCfg<D>::RS;
  const int m = h.hi_m, L = h.L;
  int T = 1;
  for (int k = 0; k < m; ++k) T *= D;
  const int S = h.srow[L - m];  // d^(L-1-m): row stride of the lowest top mode
  if constexpr (D % 2 == 0) {
    for (int e = threadIdx.x; e < T * D / 2; e += kBlock) {
      const int lr = e / (D / 2), c = e % (D / 2);
      reinterpret_cast<float4 *>(tile + lr * RS)[c] =
          reinterpret_cast<const float4 *>(psi + ((size_t)t + (size_t)lr * S) * D)[c];
    }
  } else {
    for (int e = threadIdx.x; e < T * D; e += kBlock)
      tile[(e / D) * RS + e % D] = psi[((size_t)t + (size_t)(e / D) * S) * D + e % D];
  }
  __syncthreads();
  const float J = h.J, Dl = h.Delta;
  for (int lr = threadIdx.x; lr < T; lr += kBlock) {
    float2 acc[D];
#pragma unroll
    for (int q = 0; q < D; ++q) acc[q] = make_float2(0.f, 0.f);
    int dg[kMaxL];
    {
      int u = lr;
      for (int k = 0; k < m; ++k) {
        dg[k] = u % D;
        u /= D;
      }
    }
    // bonds (L-m+k-1, L-m+k), k = 1..m-1, local strides D^(k-1), D^k
    int si = 1;
    for (int k = 1; k < m; ++k) {
      const int sj = si * D;
      const int ni = dg[k - 1], nj = dg[k];
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
      si = sj;
    }
    // ring bond (0, L-1): mode 0 inside the row, mode L-1 = local digit m-1
    if (h.periodic_wrap) {
      const int nj = dg[m - 1], sj = si;  // si = D^(m-1) here
      if (nj <= D - 2) {
        float2 P[D];
        lds_row<D>(tile, lr + sj, P);
        const float spj = sqrtf((float)nj + 1.f);
        if (J != 0.f) {
          const float c = -J * spj;
#pragma unroll
          for (int q = 1; q < D; ++q) {
            acc[q].x = fmaf(c * h.sq[q], P[q - 1].x, acc[q].x);
            acc[q].y = fmaf(c * h.sq[q], P[q - 1].y, acc[q].y);
          }
        }
        if (Dl != 0.f) {
          const float c = Dl * spj;
#pragma unroll
          for (int q = 0; q < D - 1; ++q) {
            acc[q].x = fmaf(c * h.sq[q + 1], P[q + 1].x, acc[q].x);
            acc[q].y = fmaf(c * h.sq[q + 1], P[q + 1].y, acc[q].y);
          }
        }
      }
      if (nj >= 1) {
        float2 Mv[D];
        lds_row<D>(tile, lr - sj, Mv);
        const float smj = sqrtf((float)nj);
        if (J != 0.f) {
          const float c = -J * smj;
#pragma unroll
          for (int q = 0; q < D - 1; ++q) {
            acc[q].x = fmaf(c * h.sq[q + 1], Mv[q + 1].x, acc[q].x);
            acc[q].y = fmaf(c * h.sq[q + 1], Mv[q + 1].y, acc[q].y);
          }
        }
        if (Dl != 0.f) {
          const float c = Dl * smj;
#pragma unroll
          for (int q = 1; q < D; ++q) {
            acc[q].x = fmaf(c * h.sq[q], Mv[q - 1].x, acc[q].x);
            acc[q].y = fmaf(c * h.sq[q], Mv[q - 1].y, acc[q].y);
          }
        }
      }
    }
    store_row<D>(hpsi + ((size_t)t + (size_t)lr * S) * D, acc);
  }
  __syncthreads();
}

// ---------------------------------------------------------------- lane-split stencil (d = 8, open chains)
// Four lanes share a row, two amplitudes each (c = t % 4 owns n_0 = 2c, 2c+1).
// Tile: the 512 rows with n_1..n_3 free (32 kB of LDS, unpadded; the rows a
// wavefront touches at one offset are 16 consecutive rows, 1 kB contiguous).
// Thread t owns the rows with n_1 + 8 n_2 = t / 4 and walks n_3 = p = 0..7,
// so within a wavefront n_3 and the tile's digits n_4..n_{L-1} are uniform:
// the bonds (3,4) .. (L-2, L-1) read 1 kB blocks of rows from global memory
// at wavefront-uniform offsets with wavefront-uniform coefficients and
// validity, and the lane coefficients of the bonds (0,1), (1,2) and the lane
// half of (2,3) are computed once per thread.  Terms and signs as in hblock.
constexpr int kLanesTileF4 = 2048;  // float4 words of a tile: 512 rows x 8 amplitudes
constexpr int kLanesMinL = 4, kLanesMaxL = 10;

__device__ __forceinline__ void fma4(float4 &acc, float c, const float4 &v) {
  acc.x = fmaf(c, v.x, acc.x);
  acc.y = fmaf(c, v.y, acc.y);
  acc.z = fmaf(c, v.z, acc.z);
  acc.w = fmaf(c, v.w, acc.w);
}

template <int L>
__device__ __forceinline__ void hblock_lanes8(int vb, const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                              const HamArgs &h, float4 *tile, float &e_out, float &nn_out) {
  static_assert(L >= kLanesMinL && L <= kLanesMaxL, "lane-split stencil: 4 <= L <= 10");
  constexpr int NB = L - 4;  // bonds (r-1, r), r = 4..L-1, whose neighbours lie outside the tile
  constexpr int NBA = NB > 0 ? NB : 1;  // array extent
  const float4 *__restrict__ g4 = reinterpret_cast<const float4 *>(psi);
  float4 *__restrict__ o4 = reinterpret_cast<float4 *>(hpsi);
  const float2 *tile2 = reinterpret_cast<const float2 *>(tile);
  const size_t tb = (size_t)vb * kLanesTileF4;
  for (int e = threadIdx.x; e < kLanesTileF4; e += kBlock) tile[e] = g4[tb + e];

  const float J = h.J, Dl = h.Delta, c2 = h.c2, mu = h.mu;
  auto fdiag = [&](float n) { return c2 * n * (n - 1.f) - mu * n; };
  // tile digits n_4..n_{L-1} (wavefront-uniform) and their diagonal share
  int hd[L + 1];
  float dtile = 0.f;
  {
    uint32_t v = (uint32_t)vb;
#pragma unroll
    for (int r = 4; r < L; ++r) {
      hd[r] = (int)(v & 7u);
      v >>= 3;
      dtile += fdiag((float)hd[r]);
    }
  }
  // bonds (r-1, r), r >= 5: tile-uniform validity, float4 offsets, coefficients
  bool ev[NBA][4];
  int eo[NBA][4];
  float ec[NBA][4];
#pragma unroll
  for (int b = 1; b < NB; ++b) {
    const int r = b + 4, ni = hd[r - 1], nj = hd[r];
    const int si = 4 << (3 * (r - 2)), sj = 4 << (3 * (r - 1));  // mode strides in float4 words
    const float smi = sqrtf((float)ni), spi = sqrtf((float)ni + 1.f);
    const float smj = sqrtf((float)nj), spj = sqrtf((float)nj + 1.f);
    ev[b][0] = ni >= 1 && nj <= 6; eo[b][0] = -si + sj; ec[b][0] = -J * smi * spj;
    ev[b][1] = ni <= 6 && nj >= 1; eo[b][1] = si - sj;  ec[b][1] = -J * spi * smj;
    ev[b][2] = ni <= 6 && nj <= 6; eo[b][2] = si + sj;  ec[b][2] = Dl * spi * spj;
    ev[b][3] = ni >= 1 && nj >= 1; eo[b][3] = -si - sj; ec[b][3] = Dl * smi * smj;
  }
  float s4m = 0.f, s4p = 0.f;
  if constexpr (L > 4) {
    s4m = sqrtf((float)hd[4]);
    s4p = sqrtf((float)hd[4] + 1.f);
  }

  // lane-fixed part
  const int t = threadIdx.x, c = t & 3, rip = t >> 2, n1 = rip & 7, n2 = rip >> 3;
  const float s1m = sqrtf((float)n1), s1p = sqrtf((float)n1 + 1.f);
  const float s2m = sqrtf((float)n2), s2p = sqrtf((float)n2 + 1.f);
  const float sq0 = sqrtf((float)(2 * c)), sq1 = sqrtf((float)(2 * c + 1)), sq2 = sqrtf((float)(2 * c + 2));
  // bond (0,1): rows n_1 + 1 (P) and n_1 - 1 (M), shifted by one amplitude
  const bool vP = n1 <= 6, vM = n1 >= 1;
  const float cPJ0 = vP ? -J * s1p * sq0 : 0.f;             // P[2c-1] -> n_0 = 2c
  const float cPJ1 = vP ? -J * s1p * sq1 : 0.f;             // P[2c]   -> 2c+1
  const float cPD0 = vP ? Dl * s1p * sq1 : 0.f;             // P[2c+1] -> 2c
  const float cPD1 = (vP && c < 3) ? Dl * s1p * sq2 : 0.f;  // P[2c+2] -> 2c+1
  const float cMJ0 = vM ? -J * s1m * sq1 : 0.f;             // M[2c+1] -> 2c
  const float cMJ1 = (vM && c < 3) ? -J * s1m * sq2 : 0.f;  // M[2c+2] -> 2c+1
  const float cMD0 = vM ? Dl * s1m * sq0 : 0.f;             // M[2c-1] -> 2c
  const float cMD1 = vM ? Dl * s1m * sq1 : 0.f;             // M[2c]   -> 2c+1
  const int oP = vP ? 4 : 0, oM = vM ? -4 : 0;              // float4 offsets of the rows n_1 +- 1
  const int sm1 = c > 0 ? -1 : 0, sp2 = c < 3 ? 2 : 1;      // float2 offsets of amplitudes 2c-1, 2c+2 (clamped)
  // bond (1,2): lane-fixed
  float c12[4];
  int o12[4];
  {
    const bool a0 = n1 >= 1 && n2 <= 6, a1 = n1 <= 6 && n2 >= 1, a2 = n1 <= 6 && n2 <= 6, a3 = n1 >= 1 && n2 >= 1;
    c12[0] = a0 ? -J * s1m * s2p : 0.f; o12[0] = a0 ? 4 * 7 : 0;
    c12[1] = a1 ? -J * s1p * s2m : 0.f; o12[1] = a1 ? -4 * 7 : 0;
    c12[2] = a2 ? Dl * s1p * s2p : 0.f; o12[2] = a2 ? 4 * 9 : 0;
    c12[3] = a3 ? Dl * s1m * s2m : 0.f; o12[3] = a3 ? -4 * 9 : 0;
  }
  // bond (2,3): lane half of the coefficients (times sqrt of n_3 or n_3 + 1 per pass)
  float l23[4];
  int o23[4];
  {
    const bool b_m = n2 >= 1, b_p = n2 <= 6;
    l23[0] = b_m ? -J * s2m : 0.f; o23[0] = b_m ? 4 * 56 : 0;   // n_2 - 1, n_3 + 1
    l23[1] = b_p ? -J * s2p : 0.f; o23[1] = b_p ? -4 * 56 : 0;  // n_2 + 1, n_3 - 1
    l23[2] = b_p ? Dl * s2p : 0.f; o23[2] = b_p ? 4 * 72 : 0;   // n_2 + 1, n_3 + 1
    l23[3] = b_m ? Dl * s2m : 0.f; o23[3] = b_m ? -4 * 72 : 0;  // n_2 - 1, n_3 - 1
  }
  const float dl0 = fdiag((float)n1) + fdiag((float)n2) + fdiag((float)(2 * c));
  const float dl1 = fdiag((float)n1) + fdiag((float)n2) + fdiag((float)(2 * c + 1));
  __syncthreads();

  float e = 0.f, nn = 0.f;
  const float4 *__restrict__ gt = g4 + tb;  // this tile's first word (wavefront-uniform)
  const uint32_t ut = (uint32_t)t;
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    // p is a compile-time constant after unrolling: sqrt(n_3), validity of n_3 +- 1
    const float smp = sqrtf((float)p), spp = sqrtf((float)p + 1.f);
    const int w = p * 256 + t;  // this thread's float4 word in the tile
    // bonds leaving the tile: all loads first, each under a wavefront-uniform
    // validity test (the same test guards its use below)
    float4 gv[NBA][4];
    bool gvv[NBA][4];
    if constexpr (L > 4) {
      const int nj = hd[4];
      gvv[0][0] = p >= 1 && nj <= 6;
      gvv[0][1] = p <= 6 && nj >= 1;
      gvv[0][2] = p <= 6 && nj <= 6;
      gvv[0][3] = p >= 1 && nj >= 1;
      const int o0[4] = {-256 + 2048, 256 - 2048, 256 + 2048, -256 - 2048};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (gvv[0][k]) gv[0][k] = (gt + (p * 256 + o0[k]))[ut];
    }
#pragma unroll
    for (int b = 1; b < NB; ++b)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        gvv[b][k] = ev[b][k];
        if (gvv[b][k]) gv[b][k] = (gt + (p * 256 + eo[b][k]))[ut];
      }
    const float4 own = tile[w];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    // bond (0,1)
    {
      const float4 P = tile[w + oP], M = tile[w + oM];
      const float2 Pm = tile2[2 * (w + oP) + sm1], Pp = tile2[2 * (w + oP) + sp2];
      const float2 Mm = tile2[2 * (w + oM) + sm1], Mp = tile2[2 * (w + oM) + sp2];
      acc.x = fmaf(cPJ0, Pm.x, acc.x); acc.y = fmaf(cPJ0, Pm.y, acc.y);
      acc.x = fmaf(cPD0, P.z, acc.x);  acc.y = fmaf(cPD0, P.w, acc.y);
      acc.x = fmaf(cMJ0, M.z, acc.x);  acc.y = fmaf(cMJ0, M.w, acc.y);
      acc.x = fmaf(cMD0, Mm.x, acc.x); acc.y = fmaf(cMD0, Mm.y, acc.y);
      acc.z = fmaf(cPJ1, P.x, acc.z);  acc.w = fmaf(cPJ1, P.y, acc.w);
      acc.z = fmaf(cPD1, Pp.x, acc.z); acc.w = fmaf(cPD1, Pp.y, acc.w);
      acc.z = fmaf(cMJ1, Mp.x, acc.z); acc.w = fmaf(cMJ1, Mp.y, acc.w);
      acc.z = fmaf(cMD1, M.x, acc.z);  acc.w = fmaf(cMD1, M.y, acc.w);
    }
    // bond (1,2)
#pragma unroll
    for (int k = 0; k < 4; ++k) fma4(acc, c12[k], tile[w + o12[k]]);
    // bond (2,3)
    if (p <= 6) {
      fma4(acc, l23[0] * spp, tile[w + o23[0]]);
      fma4(acc, l23[2] * spp, tile[w + o23[2]]);
    }
    if (p >= 1) {
      fma4(acc, l23[1] * smp, tile[w + o23[1]]);
      fma4(acc, l23[3] * smp, tile[w + o23[3]]);
    }
    // bonds leaving the tile
    if constexpr (L > 4) {
      const float c0[4] = {-J * smp * s4p, -J * spp * s4m, Dl * spp * s4p, Dl * smp * s4m};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (gvv[0][k]) fma4(acc, c0[k], gv[0][k]);
    }
#pragma unroll
    for (int b = 1; b < NB; ++b)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (gvv[b][k]) fma4(acc, ec[b][k], gv[b][k]);
    // diagonal, energy and norm
    const float dp = dtile + fdiag((float)p);
    const float dg0 = dp + dl0, dg1 = dp + dl1;
    acc.x = fmaf(dg0, own.x, acc.x);
    acc.y = fmaf(dg0, own.y, acc.y);
    acc.z = fmaf(dg1, own.z, acc.z);
    acc.w = fmaf(dg1, own.w, acc.w);
    e = fmaf(own.x, acc.x, fmaf(own.y, acc.y, e));
    e = fmaf(own.z, acc.z, fmaf(own.w, acc.w, e));
    nn = fmaf(own.x, own.x, fmaf(own.y, own.y, nn));
    nn = fmaf(own.z, own.z, fmaf(own.w, own.w, nn));
    (o4 + tb + p * 256)[ut] = acc;
  }
  e_out = e;
  nn_out = nn;
  __syncthreads();
}

// ---------------------------------------------------------------- pool scoring (Eq. grad)
// z += conj(a) * b
__device__ __forceinline__ void cdot_acc(float &zr, float &zi, float2 a, float2 b) {
  zr = fmaf(a.x, b.x, fmaf(a.y, b.y, zr));
  zi = fmaf(a.x, b.y, fmaf(-a.y, b.x, zi));
}

__device__ __forceinline__ int digit_of(uint64_t lo, uint64_t hi, int r) {
  return (int)((r < 16 ? (lo >> (4 * r)) : (hi >> (4 * (r - 16)))) & 15ull);
}

// Same LDS tiling as the Hamiltonian stencil: psi rows with digits n_1..n_K
// varying fully are staged in LDS (padded row stride), pairs inside modes
// 0..K read their neighbours there, wider pairs read rows from global memory.
// Each thread owns up to two rows of the tile (tiles have at most 512 rows).
template <int D>
struct PTile {
  static constexpr int RS = (D % 2 == 0) ? D + 2 : D + 1;
  static constexpr int MAXROWS = (4096 / D) < 512 ? (4096 / D) : 512;
};

template <int D>
__device__ __forceinline__ void prow(const float2 *tile, int r, float2 (&v)[D]) {
  constexpr int RS = PTile<D>::RS;
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
__device__ __forceinline__ void nbr_row(const float2 *tile, const float2 *__restrict__ psi, bool in_tile, int lr,
                                        int row, int off, float2 (&v)[D]) {
  if (in_tile) prow<D>(tile, lr + off, v);
  else load_row<D>(psi + (size_t)(row + off) * D, v);
}

template <int D>
__device__ __forceinline__ void hdot(const float2 (&h)[D], const float2 (&v)[D], float &zr, float &zi) {
  float r = 0.f, im = 0.f;
#pragma unroll
  for (int q = 0; q < D; ++q) cdot_acc(r, im, h[q], v[q]);
  zr = r;
  zi = im;
}

// Work of tile vb: this tile's share of every pool gradient, written to
// partial[vb * nslots + slot].  tile: PTile<D>::MAXROWS * RS float2 of LDS;
// acc: 4 x kMaxSlots doubles of LDS.  Contains barriers.
template <int D>
__device__ __forceinline__ void pool_block(int vb, const float2 *__restrict__ psi, const float2 *__restrict__ hpsi,
                                           double *__restrict__ partial, const PoolArgs &a,
                                           const PoolPair *__restrict__ pairs, const PoolDiag *__restrict__ diags,
                                           float2 *tile, double (*acc)[kMaxSlots]) {
  constexpr int RS = PTile<D>::RS;
  for (int k = threadIdx.x; k < 4 * kMaxSlots; k += kBlock) (&acc[0][0])[k] = 0.0;
  int K = 0, T = 1;
  while (K < a.L - 1 && T * D <= PTile<D>::MAXROWS) {
    T *= D;
    ++K;
  }
  const int r0 = vb * T;
  {
    const float2 *src = psi + (size_t)r0 * D;
    if constexpr (D % 2 == 0) {
      const float4 *s4 = reinterpret_cast<const float4 *>(src);
      for (int e = threadIdx.x; e < T * D / 2; e += kBlock)
        reinterpret_cast<float4 *>(tile + (e / (D / 2)) * RS)[e % (D / 2)] = s4[e];
    } else {
      for (int e = threadIdx.x; e < T * D; e += kBlock) tile[(e / D) * RS + e % D] = src[e];
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // this thread's rows (at most two) and their digits
  float2 h[2][D];
  uint64_t lo[2] = {0, 0}, hi[2] = {0, 0};
  int lrs[2] = {-1, -1};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int lr = threadIdx.x + k * kBlock;
    if (lr < T) {
      lrs[k] = lr;
      load_row<D>(hpsi + (size_t)(r0 + lr) * D, h[k]);
      uint32_t t = (uint32_t)(r0 + lr);
      for (int r = 1; r < a.L; ++r) {
        const uint64_t dg = t % D;
        t /= D;
        if (r < 16) lo[k] |= dg << (4 * r);
        else hi[k] |= dg << (4 * (r - 16));
      }
    } else {
#pragma unroll
      for (int q = 0; q < D; ++q) h[k][q] = make_float2(0.f, 0.f);
    }
  }

  for (int p = 0; p < a.npairs; ++p) {
    const PoolPair pp = pairs[p];
    const bool needX = pp.slot[0] >= 0 || pp.slot[1] >= 0 || pp.slot[2] >= 0;
    const bool needY = pp.slot[3] >= 0 || pp.slot[4] >= 0;
    const int i = pp.i, j = pp.j;
    const bool in_tile = j <= K;
    const int sj = a.srow[j];
    float vals[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (lrs[k] < 0) continue;
      const int lr = lrs[k], row = r0 + lr;
      float x1r = 0.f, x1i = 0.f, x2r = 0.f, x2i = 0.f, xdi = 0.f, y1r = 0.f, y1i = 0.f, y2r = 0.f, y2i = 0.f;
      const int nj = digit_of(lo[k], hi[k], j);
      float2 v[D];
      if (i >= 1) {
        // all neighbour rows of the pair are loaded unconditionally (an invalid
        // neighbour reads the row itself with weight 0) so they are in flight together
        const int ni = digit_of(lo[k], hi[k], i);
        const int si = a.srow[i];
        const float smi = sqrtf((float)ni), spi = sqrtf((float)ni + 1.f), smj = sqrtf((float)nj),
                    spj = sqrtf((float)nj + 1.f);
        const bool v0 = ni >= 1 && nj <= D - 2, v1 = ni <= D - 2 && nj >= 1;
        const bool v2 = ni <= D - 2 && nj <= D - 2, v3 = ni >= 1 && nj >= 1;
        const float c0 = v0 ? smi * spj : 0.f, c1 = v1 ? spi * smj : 0.f;
        const float c2 = v2 ? spi * spj : 0.f, c3 = v3 ? smi * smj : 0.f;
        float2 w0[D], w1[D], w2[D], w3[D];
        if (needX) {
          nbr_row<D>(tile, psi, in_tile, lr, row, v0 ? -si + sj : 0, w0);
          nbr_row<D>(tile, psi, in_tile, lr, row, v1 ? si - sj : 0, w1);
        }
        if (needY) {
          nbr_row<D>(tile, psi, in_tile, lr, row, v2 ? si + sj : 0, w2);
          nbr_row<D>(tile, psi, in_tile, lr, row, v3 ? -si - sj : 0, w3);
        }
        float zr, zi;
        if (needX) {
          hdot<D>(h[k], w0, zr, zi);
          x1r = c0 * zr;
          x1i = c0 * zi;
          hdot<D>(h[k], w1, zr, zi);
          x2r = c1 * zr;
          x2i = c1 * zi;
          xdi = (float)ni * x1i + (float)(ni + 1) * x2i;
        }
        if (needY) {
          hdot<D>(h[k], w2, zr, zi);
          y1r = c2 * zr;
          y1i = c2 * zi;
          hdot<D>(h[k], w3, zr, zi);
          y2r = c3 * zr;
          y2i = c3 * zi;
        }
      } else {
        if (nj <= D - 2) {
          nbr_row<D>(tile, psi, in_tile, lr, row, sj, v);
          const float spj = sqrtf((float)nj + 1.f);
          if (needX) {  // a_0^+ a_j: conj(h[q]) sqrt(q) v[q-1]; DH weight n_0 = q
            float r = 0.f, im = 0.f, rd = 0.f;
#pragma unroll
            for (int q = 1; q < D; ++q) {
              float zr = 0.f, zi = 0.f;
              cdot_acc(zr, zi, h[k][q], v[q - 1]);
              r = fmaf(a.sq[q], zr, r);
              im = fmaf(a.sq[q], zi, im);
              rd = fmaf((float)q * a.sq[q], zi, rd);
            }
            x1r = spj * r;
            x1i = spj * im;
            xdi += spj * rd;
          }
          if (needY) {  // a_0 a_j: conj(h[q]) sqrt(q+1) v[q+1]
            float r = 0.f, im = 0.f;
#pragma unroll
            for (int q = 0; q < D - 1; ++q) {
              float zr = 0.f, zi = 0.f;
              cdot_acc(zr, zi, h[k][q], v[q + 1]);
              r = fmaf(a.sq[q + 1], zr, r);
              im = fmaf(a.sq[q + 1], zi, im);
            }
            y1r = spj * r;
            y1i = spj * im;
          }
        }
        if (nj >= 1) {
          nbr_row<D>(tile, psi, in_tile, lr, row, -sj, v);
          const float smj = sqrtf((float)nj);
          if (needX) {  // a_j^+ a_0: conj(h[q]) sqrt(q+1) v[q+1]; DH weight n_0 + 1 = q + 1
            float r = 0.f, im = 0.f, rd = 0.f;
#pragma unroll
            for (int q = 0; q < D - 1; ++q) {
              float zr = 0.f, zi = 0.f;
              cdot_acc(zr, zi, h[k][q], v[q + 1]);
              r = fmaf(a.sq[q + 1], zr, r);
              im = fmaf(a.sq[q + 1], zi, im);
              rd = fmaf((float)(q + 1) * a.sq[q + 1], zi, rd);
            }
            x2r = smj * r;
            x2i = smj * im;
            xdi += smj * rd;
          }
          if (needY) {  // a_0^+ a_j^+: conj(h[q]) sqrt(q) v[q-1]
            float r = 0.f, im = 0.f;
#pragma unroll
            for (int q = 1; q < D; ++q) {
              float zr = 0.f, zi = 0.f;
              cdot_acc(zr, zi, h[k][q], v[q - 1]);
              r = fmaf(a.sq[q], zr, r);
              im = fmaf(a.sq[q], zi, im);
            }
            y2r = smj * r;
            y2i = smj * im;
          }
        }
      }
      vals[0] += 2.f * (x1r - x2r);
      vals[1] += -2.f * (x1i + x2i);
      vals[2] += -2.f * xdi;
      vals[3] += 2.f * (y1r - y2r);
      vals[4] += -2.f * (y1i + y2i);
    }
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      if (pp.slot[t] >= 0) {
        const float v = wave_sum_f(vals[t]);
        if (lane == 0) acc[wave][pp.slot[t]] += (double)v;
      }
    }
  }

  for (int kd = 0; kd < a.ndiag; ++kd) {
    const PoolDiag pd = diags[kd];
    float v = 0.f;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (lrs[k] < 0) continue;
      float2 own[D];
      prow<D>(tile, lrs[k], own);
      // -2 f(n) Im(conj(h) psi), f = n_r^2 (KERR), n_r (ROT) or n_r n_r2 (CK, r < r2)
      const int m2 = pd.type == FOCK_CK ? digit_of(lo[k], hi[k], pd.r2) : 1;  // r2 >= 1: a row digit
      if (pd.r == 0) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const float f = pd.type == FOCK_KERR ? (float)(q * q) : (float)(q * m2);
          v = fmaf(f, h[k][q].x * own[q].y - h[k][q].y * own[q].x, v);
        }
      } else {
        const int n = digit_of(lo[k], hi[k], pd.r);
        const float f = pd.type == FOCK_KERR ? (float)(n * n) : (float)(n * m2);
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < D; ++q) s = fmaf(h[k][q].x, own[q].y, fmaf(-h[k][q].y, own[q].x, s));
        v = fmaf(f, s, v);
      }
    }
    v = wave_sum_f(-2.f * v);
    if (lane == 0) acc[wave][pd.slot] += (double)v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.nslots; k += kBlock)
    partial[(size_t)vb * a.nslots + k] = (acc[0][k] + acc[1][k]) + (acc[2][k] + acc[3][k]);
  __syncthreads();
}


}  // namespace fock
