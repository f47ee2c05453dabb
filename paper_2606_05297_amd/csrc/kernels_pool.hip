// Pool scoring, Eq. (grad): g_k = 2 Re <H psi | A_k psi> for every pool entry
// in one pass over (psi, H psi).
//
// For a mode pair (i, j) all two-mode generators are built from four shifted
// neighbours of psi (Sec. II.A ladder action):
//   X1 = sum_n conj(h[n]) sqrt(n_i) sqrt(n_j+1) psi[n - e_i + e_j]     (a_i^+ a_j)
//   X2 = sum_n conj(h[n]) sqrt(n_i+1) sqrt(n_j) psi[n + e_i - e_j]     (a_j^+ a_i)
//   Y1 = sum_n conj(h[n]) sqrt(n_i+1) sqrt(n_j+1) psi[n + e_i + e_j]   (a_i a_j)
//   Y2 = sum_n conj(h[n]) sqrt(n_i) sqrt(n_j) psi[n - e_i - e_j]       (a_i^+ a_j^+)
// and, with Xd = sum_n conj(h) [n_i (a_i^+ a_j psi) + (n_i + 1)(a_j^+ a_i psi)],
//   g_HR = 2 Re(X1 - X2),  g_HI = -2 Im(X1 + X2),  g_DH = -2 Im(Xd),
//   g_PR = 2 Re(Y1 - Y2),  g_PI = -2 Im(Y1 + Y2).
// Single-mode diagonal generators A = i f(N_r) give g = -2 sum f(n_r) Im(conj(h) psi).
//
// One thread per row of d amplitudes along mode 0; per pair each thread forms
// its row's share, the wavefront reduces it (FP32 over 64 rows) and lane 0
// adds the wave total to a per-wave FP64 slot in LDS.  Each workgroup writes
// one FP64 partial per pool slot; a fixed-order reduction follows.
#include "device_common.h"

namespace fock {

// z += conj(a) * b
__device__ __forceinline__ void cdot_acc(float &zr, float &zi, float2 a, float2 b) {
  zr = fmaf(a.x, b.x, fmaf(a.y, b.y, zr));
  zi = fmaf(a.x, b.y, fmaf(-a.y, b.x, zi));
}

template <int D>
__device__ __forceinline__ void row_dot(const float2 (&h)[D], const float2 *__restrict__ p, float &zr, float &zi) {
  float2 v[D];
  load_row<D>(p, v);
  float r = 0.f, im = 0.f;
#pragma unroll
  for (int q = 0; q < D; ++q) cdot_acc(r, im, h[q], v[q]);
  zr = r;
  zi = im;
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

template <int D>
__global__ __launch_bounds__(kBlock) void k_pool(const float2 *__restrict__ psi, const float2 *__restrict__ hpsi,
                                                 double *__restrict__ partial, PoolArgs a,
                                                 const PoolPair *__restrict__ pairs,
                                                 const PoolDiag *__restrict__ diags) {
  constexpr int RS = PTile<D>::RS;
  __shared__ double acc[4][kMaxSlots];
  __shared__ float4 tile4[(PTile<D>::MAXROWS * RS + 1) / 2];
  float2 *tile = reinterpret_cast<float2 *>(tile4);
  for (int k = threadIdx.x; k < 4 * kMaxSlots; k += kBlock) (&acc[0][0])[k] = 0.0;
  int K = 0, T = 1;
  while (K < a.L - 1 && T * D <= PTile<D>::MAXROWS) {
    T *= D;
    ++K;
  }
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
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
      // -2 f(n_r) Im(conj(h) psi), f = n^2 (KERR) or n (ROT)
      if (pd.r == 0) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const float f = pd.type == FOCK_KERR ? (float)(q * q) : (float)q;
          v = fmaf(f, h[k][q].x * own[q].y - h[k][q].y * own[q].x, v);
        }
      } else {
        const int n = digit_of(lo[k], hi[k], pd.r);
        const float f = pd.type == FOCK_KERR ? (float)(n * n) : (float)n;
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
}

int pool_blocks(const PoolArgs &a) { return a.nrows / apply_h_tile_rows(a.L, a.d); }

template <int D>
static void launch_pool_t(const PoolArgs &a, const PoolPair *pairs, const PoolDiag *diags, const float2 *psi,
                          const float2 *hpsi, double *partial, int G, hipStream_t s) {
  hipLaunchKernelGGL(k_pool<D>, dim3(G), dim3(kBlock), 0, s, psi, hpsi, partial, a, pairs, diags);
}

int launch_pool(const PoolArgs &a, const PoolPair *pairs, const PoolDiag *diags, const float2 *psi,
                const float2 *hpsi, double *partial, int *nblocks, hipStream_t s) {
  const int G = pool_blocks(a);
  *nblocks = G;
  switch (a.d) {
#define CASE(D) \
  case D: launch_pool_t<D>(a, pairs, diags, psi, hpsi, partial, G, s); break;
    CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13)
    CASE(14) CASE(15) CASE(16)
#undef CASE
    default: return set_error(FOCK_ERR_UNSUPPORTED, "d=%d unsupported", a.d);
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
