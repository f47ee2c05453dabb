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
#include "stencil_kernels.h"

namespace fock {

template <int D>
__global__ __launch_bounds__(kBlock) void k_apply_h(const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                                    double *__restrict__ partial, HamArgs h) {
  __shared__ double red[4];
  __shared__ float4 tile4[TileCfg<D>::PWORDS];
  const int vb = h.order ? h.order[blockIdx.x] : xcd_remap(blockIdx.x, gridDim.x);
  float e = 0.f, nn = 0.f;
  hblock<D>(vb, psi, hpsi, h, reinterpret_cast<float2 *>(tile4), e, nn);
  const double se = block_sum_d((double)e, red);
  const double sn = block_sum_d((double)nn, red);
  if (threadIdx.x == 0) {
    partial[2 * vb] = se;
    partial[2 * vb + 1] = sn;
  }
}

// Lane-split H psi (see hblock_lanes8); same tiles and partials as k_apply_h<8>.
template <int L>
__global__ __launch_bounds__(kBlock) void k_apply_h_lanes8(const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                                           double *__restrict__ partial, HamArgs h) {
  __shared__ double red[4];
  __shared__ float4 tile4[kLanesTileF4];
  const int vb = h.order ? h.order[blockIdx.x] : xcd_remap(blockIdx.x, gridDim.x);
  float e = 0.f, nn = 0.f;
  hblock_lanes8<L>(vb, psi, hpsi, h, tile4, e, nn);
  const double se = block_sum_d((double)e, red);
  const double sn = block_sum_d((double)nn, red);
  if (threadIdx.x == 0) {
    partial[2 * vb] = se;
    partial[2 * vb + 1] = sn;
  }
}

// First pass of the two-pass stencil (see hblock_hi); tile t = workgroup's
// virtual index.
template <int D>
__global__ __launch_bounds__(kBlock) void k_apply_h_hi(const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                                       HamArgs h) {
  __shared__ float4 tile4[TileCfg<D>::PWORDS];
  hblock_hi<D>(xcd_remap(blockIdx.x, gridDim.x), psi, hpsi, h, reinterpret_cast<float2 *>(tile4));
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

// Rows 0..n-1 as k_reduce_rows into out[2 + k], and (workgroups n, n + 1) the
// two columns of the energy and norm partials epart[2 b + c], b < ne, into
// out[c]: the reduction of a whole gradient evaluation in one launch.
__global__ __launch_bounds__(kBlock) void k_reduce_rows_e(const double *__restrict__ partial, int row_stride,
                                                          const GateRec *__restrict__ recs, int n,
                                                          const double *__restrict__ epart, int ne,
                                                          double *__restrict__ out) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double s = 0.0;
  if (k < n) {
    const int nb = recs[k].nblk;
    for (int b = threadIdx.x; b < nb; b += kBlock) s += partial[(size_t)k * row_stride + b];
  } else {
    for (int b = threadIdx.x; b < ne; b += kBlock) s += epart[(size_t)b * 2 + (k - n)];
  }
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) out[k < n ? 2 + k : k - n] = s;
}

int launch_reduce_rows_energy(const double *partial, int row_stride, const GateRec *recs, int n,
                              const double *epart, int ne, double *out, hipStream_t s) {
  if (n < 0 || ne <= 0) return set_error(FOCK_ERR_ARG, "reduction of %d rows and %d energy partials", n, ne);
  hipLaunchKernelGGL(k_reduce_rows_e, dim3(n + 2), dim3(kBlock), 0, s, partial, row_stride, recs, n, epart, ne, out);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
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

// Number of top modes the first pass of the two-pass stencil stages in LDS:
// the most with d^m rows fitting the tile and not reaching the single-pass
// tile's modes 0..K; 0 when that leaves no bond to take over.
int apply_h_hi_modes(int L, int d, int periodic_wrap) {
  const int T = apply_h_tile_rows(L, d);
  int K = 0;
  for (int t = 1; t < T; t *= d) ++K;
  const int maxrows = (4096 / d) < 512 ? (4096 / d) : 512;
  int m = 0;
  for (int t = d; t <= maxrows && m < L - 1 - K; t *= d) ++m;
  if (m < 2 && !(m == 1 && periodic_wrap)) return 0;
  return m;
}

template <int D>
static void launch_h_t(const HamArgs &h, const float2 *psi, float2 *hpsi, double *partial, int G, hipStream_t s) {
  if (h.hi_m > 0) {
    int GA = 1;
    for (int r = 1; r < h.L - h.hi_m; ++r) GA *= h.d;
    hipLaunchKernelGGL(k_apply_h_hi<D>, dim3(GA), dim3(kBlock), 0, s, psi, hpsi, h);
  }
  if constexpr (D == 8) {
    if (h.lanes) {
      switch (h.L) {
#define LCASE(LL) \
  case LL: hipLaunchKernelGGL(k_apply_h_lanes8<LL>, dim3(G), dim3(kBlock), 0, s, psi, hpsi, partial, h); return;
        LCASE(4) LCASE(5) LCASE(6) LCASE(7) LCASE(8) LCASE(9) LCASE(10)
#undef LCASE
        default: break;
      }
    }
  }
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
