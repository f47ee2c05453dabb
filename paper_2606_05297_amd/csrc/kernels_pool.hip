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

template <int D>
__global__ __launch_bounds__(kBlock) void k_pool(const float2 *__restrict__ psi, const float2 *__restrict__ hpsi,
                                                 double *__restrict__ partial, PoolArgs a,
                                                 const PoolPair *__restrict__ pairs,
                                                 const PoolDiag *__restrict__ diags) {
  __shared__ double acc[4][kMaxSlots];
  for (int k = threadIdx.x; k < 4 * kMaxSlots; k += kBlock) (&acc[0][0])[k] = 0.0;
  __syncthreads();
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const int row = vb * kBlock + threadIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool active = row < a.nrows;
  float2 h[D];
  uint64_t lo = 0, hi = 0;
  if (active) {
    load_row<D>(hpsi + (size_t)row * D, h);
    uint32_t t = (uint32_t)row;
    for (int r = 1; r < a.L; ++r) {
      const uint64_t dg = t % D;
      t /= D;
      if (r < 16) lo |= dg << (4 * r);
      else hi |= dg << (4 * (r - 16));
    }
  } else {
#pragma unroll
    for (int q = 0; q < D; ++q) h[q] = make_float2(0.f, 0.f);
  }

  for (int p = 0; p < a.npairs; ++p) {
    const PoolPair pp = pairs[p];
    const bool needX = pp.slot[0] >= 0 || pp.slot[1] >= 0 || pp.slot[2] >= 0;
    const bool needY = pp.slot[3] >= 0 || pp.slot[4] >= 0;
    float x1r = 0.f, x1i = 0.f, x2r = 0.f, x2i = 0.f, xdi = 0.f, y1r = 0.f, y1i = 0.f, y2r = 0.f, y2i = 0.f;
    if (active) {
      const int j = pp.j, i = pp.i;
      const int nj = digit_of(lo, hi, j);
      const int sj = a.srow[j];
      if (i >= 1) {
        const int ni = digit_of(lo, hi, i);
        const int si = a.srow[i];
        const float smi = sqrtf((float)ni), spi = sqrtf((float)ni + 1.f), smj = sqrtf((float)nj),
                    spj = sqrtf((float)nj + 1.f);
        if (needX) {
          if (ni >= 1 && nj <= D - 2) {
            float zr, zi;
            row_dot<D>(h, psi + (size_t)(row - si + sj) * D, zr, zi);
            const float c = smi * spj;
            x1r = c * zr;
            x1i = c * zi;
          }
          if (ni <= D - 2 && nj >= 1) {
            float zr, zi;
            row_dot<D>(h, psi + (size_t)(row + si - sj) * D, zr, zi);
            const float c = spi * smj;
            x2r = c * zr;
            x2i = c * zi;
          }
          xdi = (float)ni * x1i + (float)(ni + 1) * x2i;
        }
        if (needY) {
          if (ni <= D - 2 && nj <= D - 2) {
            float zr, zi;
            row_dot<D>(h, psi + (size_t)(row + si + sj) * D, zr, zi);
            const float c = spi * spj;
            y1r = c * zr;
            y1i = c * zi;
          }
          if (ni >= 1 && nj >= 1) {
            float zr, zi;
            row_dot<D>(h, psi + (size_t)(row - si - sj) * D, zr, zi);
            const float c = smi * smj;
            y2r = c * zr;
            y2i = c * zi;
          }
        }
      } else {
        // i = 0: per-position factors along the row
        if (nj <= D - 2) {
          float2 P[D];
          load_row<D>(psi + (size_t)(row + sj) * D, P);
          const float spj = sqrtf((float)nj + 1.f);
          if (needX) {  // a_0^+ a_j: conj(h[q]) sqrt(q) P[q-1]
            float r = 0.f, im = 0.f, rd = 0.f;
#pragma unroll
            for (int q = 1; q < D; ++q) {
              float zr = 0.f, zi = 0.f;
              cdot_acc(zr, zi, h[q], P[q - 1]);
              r = fmaf(a.sq[q], zr, r);
              im = fmaf(a.sq[q], zi, im);
              rd = fmaf((float)q * a.sq[q], zi, rd);
            }
            x1r = spj * r;
            x1i = spj * im;
            xdi += spj * rd;
          }
          if (needY) {  // a_0 a_j: conj(h[q]) sqrt(q+1) P[q+1]
            float r = 0.f, im = 0.f;
#pragma unroll
            for (int q = 0; q < D - 1; ++q) {
              float zr = 0.f, zi = 0.f;
              cdot_acc(zr, zi, h[q], P[q + 1]);
              r = fmaf(a.sq[q + 1], zr, r);
              im = fmaf(a.sq[q + 1], zi, im);
            }
            y1r = spj * r;
            y1i = spj * im;
          }
        }
        if (nj >= 1) {
          float2 M[D];
          load_row<D>(psi + (size_t)(row - sj) * D, M);
          const float smj = sqrtf((float)nj);
          if (needX) {  // a_j^+ a_0: conj(h[q]) sqrt(q+1) M[q+1]; DH weight n_0 + 1 = q + 1
            float r = 0.f, im = 0.f, rd = 0.f;
#pragma unroll
            for (int q = 0; q < D - 1; ++q) {
              float zr = 0.f, zi = 0.f;
              cdot_acc(zr, zi, h[q], M[q + 1]);
              r = fmaf(a.sq[q + 1], zr, r);
              im = fmaf(a.sq[q + 1], zi, im);
              rd = fmaf((float)(q + 1) * a.sq[q + 1], zi, rd);
            }
            x2r = smj * r;
            x2i = smj * im;
            xdi += smj * rd;
          }
          if (needY) {  // a_0^+ a_j^+: conj(h[q]) sqrt(q) M[q-1]
            float r = 0.f, im = 0.f;
#pragma unroll
            for (int q = 1; q < D; ++q) {
              float zr = 0.f, zi = 0.f;
              cdot_acc(zr, zi, h[q], M[q - 1]);
              r = fmaf(a.sq[q], zr, r);
              im = fmaf(a.sq[q], zi, im);
            }
            y2r = smj * r;
            y2i = smj * im;
          }
        }
      }
    }
    float vals[5];
    vals[0] = 2.f * (x1r - x2r);
    vals[1] = -2.f * (x1i + x2i);
    vals[2] = -2.f * xdi;
    vals[3] = 2.f * (y1r - y2r);
    vals[4] = -2.f * (y1i + y2i);
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      if (pp.slot[t] >= 0) {
        const float v = wave_sum_f(vals[t]);
        if (lane == 0) acc[wave][pp.slot[t]] += (double)v;
      }
    }
  }

  if (a.ndiag > 0) {
    float2 own[D];
    if (active) load_row<D>(psi + (size_t)row * D, own);
    for (int k = 0; k < a.ndiag; ++k) {
      const PoolDiag pd = diags[k];
      float v = 0.f;
      if (active) {
        // Im(conj(h) psi) weighted by f(n_r), f = n^2 (KERR) or n (ROT)
        if (pd.r == 0) {
#pragma unroll
          for (int q = 0; q < D; ++q) {
            const float f = pd.type == FOCK_KERR ? (float)(q * q) : (float)q;
            v = fmaf(f, h[q].x * own[q].y - h[q].y * own[q].x, v);
          }
        } else {
          const int n = digit_of(lo, hi, pd.r);
          const float f = pd.type == FOCK_KERR ? (float)(n * n) : (float)n;
          float s = 0.f;
#pragma unroll
          for (int q = 0; q < D; ++q) s = fmaf(h[q].x, own[q].y, fmaf(-h[q].y, own[q].x, s));
          v = f * s;
        }
      }
      v = wave_sum_f(-2.f * v);
      if (lane == 0) acc[wave][pd.slot] += (double)v;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.nslots; k += kBlock)
    partial[(size_t)vb * a.nslots + k] = (acc[0][k] + acc[1][k]) + (acc[2][k] + acc[3][k]);
}

int pool_blocks(const PoolArgs &a) { return (a.nrows + kBlock - 1) / kBlock; }

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
