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
#include "stencil_kernels.h"

namespace fock {

template <int D>
__global__ __launch_bounds__(kBlock) void k_pool(const float2 *__restrict__ psi, const float2 *__restrict__ hpsi,
                                                 double *__restrict__ partial, PoolArgs a,
                                                 const PoolPair *__restrict__ pairs,
                                                 const PoolDiag *__restrict__ diags) {
  __shared__ double acc[4][kMaxSlots];
  __shared__ float4 tile4[(PTile<D>::MAXROWS * PTile<D>::RS + 1) / 2];
  pool_block<D>(a.order ? a.order[blockIdx.x] : xcd_remap(blockIdx.x, gridDim.x), psi, hpsi, partial, a, pairs, diags,
                reinterpret_cast<float2 *>(tile4), acc);
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
