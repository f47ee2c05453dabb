// Dense two-mode gate on FP32 matrix cores: every fibre (the d^2 amplitudes
// over (n_i, n_j)) is multiplied by the full d^2 x d^2 gate matrix, as one
// real GEMM  Y[f][:] = X[f][:] W  with X[f] = (Re x_f, Im x_f) and
//   W = [[Re U^T, Im U^T], [-Im U^T, Re U^T]]  (2d^2 x 2d^2, padded to 16),
// on v_mfma_f32_16x16x4_f32.  The dense product ignores the conserved-block
// structure the block-sparse kernels exploit (Sec. II.B): at d = 8 it costs
// 512 flop per amplitude against 43, so it is the matrix-core variant of the
// same operation, kept for comparison and for small d.
//
// Persistent workgroups (one per CU: W takes 74 kB of LDS at d = 8) walk
// tiles of 64 fibres; wavefront w computes fibres 16w..16w+15 of a tile.
// MFMA lane layout (16x16x4): lane l holds A[m = l % 16][k = l / 16],
// B[k = l / 16][n = l % 16] and C[m = 4 (l / 16) + r][n = l % 16], r < 4.
#include <atomic>

#include "dense_internal.h"
#include "gate_kernels.h"

namespace fock {

GateLaunch gate_launch_params(const Geometry &g, int i, int j);

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int D>
struct DenseCfg {
  static constexpr int D2 = D * D;
  static constexpr int KP = (2 * D2 + 15) / 16 * 16;  // padded real dimension
  static constexpr int XS = KP + 4;                     // LDS row stride of X (conflict-free A reads)
  static constexpr int WS = KP + 16;                    // LDS row stride of W (conflict-free B reads)
};

// W[k][n] from the packed blocks of U (DAG: from U^+), zero outside the blocks
// and in the padding.  One thread per entry.
template <int D>
__global__ __launch_bounds__(kBlock) void k_dense_w(const float2 *__restrict__ U, int kind, int dag,
                                                    float *__restrict__ W) {
  using C = DenseCfg<D>;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= C::KP * C::KP) return;
  const int k = e / C::KP, n = e % C::KP;
  float w = 0.f;
  if (k < 2 * C::D2 && n < 2 * C::D2) {
    const int q = k % C::D2, p = n % C::D2;  // input member q, output member p
    const int ip = p / D, jp = p % D, iq = q / D, jq = q % D;
    const int sp = kind == KIND_SUM ? ip + jp : ip - jp + (D - 1);
    const int sq = kind == KIND_SUM ? iq + jq : iq - jq + (D - 1);
    if (sp == sq) {
      int off = 0;
      for (int s = 0; s < sp; ++s) {
        const int bs = blk_hi(kind, D, s) - blk_lo(kind, D, s) + 1;
        off += bs * bs;
      }
      const int lo = blk_lo(kind, D, sp), b = blk_hi(kind, D, sp) - lo + 1;
      const int pp = ip - lo, qq = iq - lo;
      float2 u = dag ? U[off + qq * b + pp] : U[off + pp * b + qq];
      if (dag) u.y = -u.y;
      // y_re[p] += Re u x_re[q] - Im u x_im[q];  y_im[p] += Im u x_re[q] + Re u x_im[q]
      const bool kim = k >= C::D2, nim = n >= C::D2;
      w = !kim && !nim ? u.x : kim && !nim ? -u.y : !kim && nim ? u.y : u.x;
    }
  }
  W[e] = w;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_gate2_dense(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                                        const float *__restrict__ Wg, GateLaunch g) {
  using C = DenseCfg<D>;
  constexpr int NF = 64;  // fibres per tile
  extern __shared__ float4 lds4[];
  float *W = reinterpret_cast<float *>(lds4);  // KP x WS
  float *X = W + C::KP * C::WS;                 // NF x XS
  for (int e = threadIdx.x; e < C::KP * C::KP; e += kBlock) W[(e / C::KP) * C::WS + e % C::KP] = Wg[e];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const uint32_t ntile = (g.nfib + NF - 1) / NF;
  const bool i0 = g.si == 1;  // pair (0, j): member n_i runs along contiguous amplitudes
  constexpr int PER = (NF * C::D2 + kBlock - 1) / kBlock;  // amplitudes per thread per tile
  // element e of a tile -> (fibre f, member q = n_i d + n_j); consecutive threads
  // take consecutive amplitudes in memory
  auto member = [&](int e, int &f, int &ni, int &nj) {
    if (i0) {
      ni = e % D;
      f = (e / D) % NF;
      nj = e / (D * NF);
    } else {
      f = e % NF;
      const int q = e / NF;
      ni = q / D;
      nj = q % D;
    }
  };
  auto gather = [&](uint32_t t, float2 (&pv)[PER]) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = threadIdx.x + k * kBlock;
      int f, ni, nj;
      member(e, f, ni, nj);
      const uint32_t fi = t * NF + (uint32_t)f;
      pv[k] = (e < NF * C::D2 && fi < g.nfib) ? src[fiber_base(fi, g, D) + ni * g.si + nj * g.sj]
                                               : make_float2(0.f, 0.f);
    }
  };
  float2 pv[PER];
  if (blockIdx.x < ntile) gather(blockIdx.x, pv);
  for (uint32_t t = blockIdx.x; t < ntile; t += gridDim.x) {
    __syncthreads();  // W ready / previous tile's stores have read X
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e < NF * C::D2) {
        int f, ni, nj;
        member(e, f, ni, nj);
        const int q = ni * D + nj;
        X[f * C::XS + q] = pv[k].x;
        X[f * C::XS + C::D2 + q] = pv[k].y;
      }
    }
    for (int e = threadIdx.x; e < NF * (C::KP - 2 * C::D2); e += kBlock) {
      const int f = e / (C::KP - 2 * C::D2), k = 2 * C::D2 + e % (C::KP - 2 * C::D2);
      X[f * C::XS + k] = 0.f;
    }
    __syncthreads();
    // the next tile's fibres are in flight while the matrix cores work on this one
    if (t + gridDim.x < ntile) gather(t + gridDim.x, pv);
    // output tiles in pairs: two independent accumulation chains per k-step
    f32x4 acc[C::KP / 16];
#pragma unroll
    for (int nt = 0; nt < C::KP / 16; nt += 2) {
      f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0;
      const bool two = nt + 1 < C::KP / 16;
#pragma unroll 8
      for (int ks = 0; ks < C::KP / 4; ++ks) {
        const float av = X[(16 * wave + lr) * C::XS + 4 * ks + lq];
        const float *wr = W + (4 * ks + lq) * C::WS + 16 * nt + lr;
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, wr[0], c0, 0, 0, 0);
        if (two) c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, wr[16], c1, 0, 0, 0);
      }
      acc[nt] = c0;
      if (two) acc[nt + 1] = c1;
    }
    __syncthreads();  // every wavefront has read X
#pragma unroll
    for (int nt = 0; nt < C::KP / 16; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) X[(16 * wave + 4 * lq + r) * C::XS + 16 * nt + lr] = acc[nt][r];
    __syncthreads();
    const uint32_t f0 = t * NF;
    for (int e = threadIdx.x; e < NF * C::D2; e += kBlock) {
      int f, ni, nj;
      member(e, f, ni, nj);
      const int q = ni * D + nj;
      if (f0 + f < g.nfib)
        dst[fiber_base(f0 + f, g, D) + ni * g.si + nj * g.sj] = make_float2(X[f * C::XS + q], X[f * C::XS + C::D2 + q]);
    }
  }
}

bool dense_supported(int d) { return d == 4 || d == 6 || d == 8; }

size_t dense_w_bytes(int d) {
  if (!dense_supported(d)) return 0;
  const int kp = (2 * d * d + 15) / 16 * 16;
  return sizeof(float) * (size_t)kp * kp;
}

#define DENSE_D_SWITCH(d, STMT)                                                                  \
  switch (d) {                                                                                   \
    case 4: { constexpr int D = 4; STMT; } break;                                                \
    case 6: { constexpr int D = 6; STMT; } break;                                                \
    case 8: { constexpr int D = 8; STMT; } break;                                                \
    default: return set_error(FOCK_ERR_UNSUPPORTED, "dense gate needs d in {4, 6, 8}, got %d", d); \
  }

int launch_gate_dense(const Geometry &geo, int i, int j, int kind, bool dag, const float2 *U, const float2 *src,
                      float2 *psi, float *W, hipStream_t s) {
  const GateLaunch gl = gate_launch_params(geo, i, j);
  DENSE_D_SWITCH(geo.d, {
    using C = DenseCfg<D>;
    hipLaunchKernelGGL(k_dense_w<D>, dim3((C::KP * C::KP + kBlock - 1) / kBlock), dim3(kBlock), 0, s, U, kind,
                       dag ? 1 : 0, W);
    const size_t lds = sizeof(float) * ((size_t)C::KP * C::WS + (size_t)64 * C::XS);
    // dynamic LDS beyond 64 kB must be allowed once per kernel and device
    static std::atomic<uint32_t> attr_set{0};
    int dev = 0;
    FOCK_HIP(hipGetDevice(&dev));
    const uint32_t bit = dev < 32 ? (1u << dev) : 0u;
    if (!bit || !(attr_set.load() & bit)) {
      FOCK_HIP(hipFuncSetAttribute((const void *)k_gate2_dense<D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
      attr_set.fetch_or(bit);
    }
    const uint32_t ntile = (gl.nfib + 63) / 64;
    const int grid = (int)(ntile < 256 ? ntile : 256);
    hipLaunchKernelGGL(k_gate2_dense<D>, dim3(grid), dim3(kBlock), lds, s, src, psi, (const float *)W, gl);
  });
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
