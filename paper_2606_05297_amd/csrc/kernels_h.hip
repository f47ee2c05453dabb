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

template <int D>
__global__ __launch_bounds__(kBlock) void k_apply_h(const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                                    double *__restrict__ partial, HamArgs h) {
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const int row = vb * kBlock + threadIdx.x;
  float e = 0.f, nn = 0.f;
  if (row < h.nrows) {
    float2 acc[D], own[D];
#pragma unroll
    for (int q = 0; q < D; ++q) acc[q] = make_float2(0.f, 0.f);
    load_row<D>(psi + (size_t)row * D, own);
    const float J = h.J, Dl = h.Delta;
    float dg_row = 0.f;
    uint32_t t = (uint32_t)row;
    int nprev = 0, n1 = 0;
    float smp = 0.f, spp = 0.f;  // sqrt(n_prev), sqrt(n_prev + 1)
    for (int r = 1; r < h.L; ++r) {
      const int n = (int)(t % D);
      t /= D;
      const float nf = (float)n;
      dg_row += h.c2 * nf * (nf - 1.f) - h.mu * nf;
      const float sm = sqrtf(nf), sp = sqrtf(nf + 1.f);
      if (r == 1) {
        n1 = n;
      } else {
        // bond (r-1, r): i = r-1, j = r, both >= 1
        const int ni = nprev, nj = n;
        const int si = h.srow[r - 1], sj = h.srow[r];
        if (J != 0.f) {
          if (ni >= 1 && nj <= D - 2) axpy_row<D>(acc, psi + (size_t)(row - si + sj) * D, -J * smp * sp);
          if (ni <= D - 2 && nj >= 1) axpy_row<D>(acc, psi + (size_t)(row + si - sj) * D, -J * spp * sm);
        }
        if (Dl != 0.f) {
          if (ni <= D - 2 && nj <= D - 2) axpy_row<D>(acc, psi + (size_t)(row + si + sj) * D, Dl * spp * sp);
          if (ni >= 1 && nj >= 1) axpy_row<D>(acc, psi + (size_t)(row - si - sj) * D, Dl * smp * sm);
        }
      }
      nprev = n;
      smp = sm;
      spp = sp;
    }
    // bonds touching mode 0: (0, 1) and the ring bond (0, L-1)
    const int nb0 = (h.L >= 2 ? 1 : 0) + h.periodic_wrap;
    for (int b = 0; b < nb0; ++b) {
      const int j = (b == 0) ? 1 : h.L - 1;
      const int nj = (b == 0) ? n1 : nprev;
      const int sj = h.srow[j];
      if (nj <= D - 2) {
        float2 P[D];
        load_row<D>(psi + (size_t)(row + sj) * D, P);
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
        load_row<D>(psi + (size_t)(row - sj) * D, M);
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

int apply_h_blocks(const HamArgs &h) { return (h.nrows + kBlock - 1) / kBlock; }

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
