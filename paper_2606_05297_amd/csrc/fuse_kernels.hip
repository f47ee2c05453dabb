// Fused gate groups: consecutive gates whose modes fit one tile of s <= 6
// modes (mode 0 always included, d^s <= 4096 amplitudes) run as one pass over
// the state.  Tile t holds the amplitudes whose digits of the tile modes take
// all values for fixed digits of the other modes; the gates of the group are
// applied one after another in LDS (Sec. II.B block form per fibre), so the
// state is read and written once per group instead of once per gate.
//
// Forward: dst <- U_k1-1 ... U_k0 src.  Reverse (adjoint sweep, Sec. IV.B
// gradient identity): for k = k1-1 .. k0, this tile's share of Re<lam|A_k phi>
// goes to partial[k * rs + t], then phi <- U_k^+ phi and lam <- U_k^+ lam.
#include "fuse_internal.h"

namespace fock {

constexpr int kFuseAmps = 4096;

// global index of local amplitude la of the tile with base `base`
__device__ __forceinline__ uint32_t fuse_gaddr(const FuseArgs &a, uint32_t base, int la, int D) {
  uint32_t g = base;
  for (int k = 0; k < a.s; ++k) {
    g += (uint32_t)(la % D) * a.tstride[k];
    la /= D;
  }
  return g;
}

__device__ __forceinline__ uint32_t fuse_base(const FuseArgs &a, int t, int D) {
  uint32_t base = 0;
  for (int k = 0; k < a.nc; ++k) {
    base += (uint32_t)(t % D) * a.cstride[k];
    t /= D;
  }
  return base;
}

// tile <-> global, pairs of amplitudes (n_0 even, n_0 + 1) as one float4
template <int D>
__device__ __forceinline__ void fuse_load(float2 *tl, const float2 *__restrict__ src, const FuseArgs &a,
                                          uint32_t base, int nt) {
  for (int w0 = 0; w0 < nt / 2; w0 += 8 * kBlock) {
    float4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int w = w0 + k * kBlock + threadIdx.x;
      v[k] = w < nt / 2 ? *reinterpret_cast<const float4 *>(src + fuse_gaddr(a, base, 2 * w, D))
                        : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int w = w0 + k * kBlock + threadIdx.x;
      if (w < nt / 2) reinterpret_cast<float4 *>(tl)[w] = v[k];
    }
  }
}

template <int D>
__device__ __forceinline__ void fuse_store(const float2 *tl, float2 *__restrict__ dst, const FuseArgs &a,
                                           uint32_t base, int nt) {
  for (int w = threadIdx.x; w < nt / 2; w += kBlock)
    *reinterpret_cast<float4 *>(dst + fuse_gaddr(a, base, 2 * w, D)) = reinterpret_cast<const float4 *>(tl)[w];
}

__device__ __forceinline__ float2 cmul(float2 m, float2 v, bool conj_m) {
  const float mi = conj_m ? -m.y : m.y;
  return make_float2(m.x * v.x - mi * v.y, m.x * v.y + mi * v.x);
}

// Local index of the first member of fibre f (digits of the positions other
// than ki, kj taken from f).
template <int D>
__device__ __forceinline__ int fuse_fbase(int f, int s, int ki, int kj) {
  int fb = 0, pw = 1;
  for (int k = 0; k < s; ++k) {
    if (k != ki && k != kj) {
      fb += (f % D) * pw;
      f /= D;
    }
    pw *= D;
  }
  return fb;
}

// Two-mode gate on tile positions (ki, kj).  Wavefront w takes the conserved
// blocks w, w+4, ... (the gate entries of a block are then uniform over the
// wavefront); its lanes take the fibres.  Each (fibre, block) maps the block's
// members through U (DAG: U^+); they touch disjoint amplitudes.
template <int D>
__device__ __forceinline__ void fuse_pair(float2 *tl, const FuseGate &g, const FuseArgs &a, int nt,
                                          const float2 *__restrict__ U, bool dag) {
  int li = 1, lj = 1;
  for (int k = 0; k < g.ki; ++k) li *= D;
  for (int k = 0; k < g.kj; ++k) lj *= D;
  constexpr int NB = 2 * D - 1;
  const int nf = nt / (D * D);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int blk = wave; blk < NB; blk += kBlock / 64) {
    const int lo = blk_lo(g.kind, D, blk), b = blk_hi(g.kind, D, blk) - lo + 1;
    const float2 *Ub = U + a.boff[blk];
    for (int f = lane; f < nf; f += 64) {
      const int fb = fuse_fbase<D>(f, a.s, g.ki, g.kj);
      int idx[D];
      float2 v[D];
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          idx[p] = fb + (lo + p) * li + blk_nj(g.kind, D, blk, lo + p) * lj;
          v[p] = tl[idx[p]];
        }
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 acc = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) {
              const float2 t = cmul(dag ? Ub[q * b + p] : Ub[p * b + q], v[q], dag);
              acc.x += t.x;
              acc.y += t.y;
            }
          tl[idx[p]] = acc;
        }
    }
  }
}

// Single-mode phase gate on tile position kr: amplitude * U[n_r] (DAG: conj).
template <int D>
__device__ __forceinline__ void fuse_diag(float2 *tl, const FuseGate &g, int nt, const float2 *__restrict__ U,
                                          bool dag) {
  int lr = 1;
  for (int k = 0; k < g.ki; ++k) lr *= D;
  for (int la = threadIdx.x; la < nt; la += kBlock) tl[la] = cmul(U[(la / lr) % D], tl[la], dag);
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_fuse_fwd(FuseArgs a, const float2 *__restrict__ src,
                                                     float2 *__restrict__ dst, const float2 *__restrict__ utab) {
  __shared__ float4 tile4[kFuseAmps / 2];
  float2 *tl = reinterpret_cast<float2 *>(tile4);
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  int nt = 1;
  for (int k = 0; k < a.s; ++k) nt *= D;
  const uint32_t base = fuse_base(a, t, D);
  fuse_load<D>(tl, src, a, base, nt);
  __syncthreads();
  for (int gi = 0; gi < a.ng; ++gi) {
    const FuseGate g = a.g[gi];
    const float2 *U = utab + g.u_off;
    if (g.kj < 0) fuse_diag<D>(tl, g, nt, U, false);
    else fuse_pair<D>(tl, g, a, nt, U, false);
    __syncthreads();
  }
  fuse_store<D>(tl, dst, a, base, nt);
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_fuse_adj(FuseArgs a, float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                     const float2 *__restrict__ utab, double *__restrict__ partial,
                                                     int rs) {
  __shared__ float4 tp4[kFuseAmps / 2], tq4[kFuseAmps / 2];
  __shared__ double red[4];
  float2 *tp = reinterpret_cast<float2 *>(tp4);  // phi
  float2 *tq = reinterpret_cast<float2 *>(tq4);  // lambda
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  int nt = 1;
  for (int k = 0; k < a.s; ++k) nt *= D;
  const uint32_t base = fuse_base(a, t, D);
  fuse_load<D>(tp, phi, a, base, nt);
  fuse_load<D>(tq, lam, a, base, nt);
  __syncthreads();
  constexpr int NB = 2 * D - 1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int gi = a.ng - 1; gi >= 0; --gi) {
    const FuseGate g = a.g[gi];
    const float2 *U = utab + g.u_off;
    // this tile's share of Re<lam|A phi>
    float gacc = 0.f;
    if (g.kj < 0) {
      int lr = 1;
      for (int k = 0; k < g.ki; ++k) lr *= D;
      for (int la = threadIdx.x; la < nt; la += kBlock) {
        const int n = (la / lr) % D;
        const float f = g.type == FOCK_KERR ? (float)(n * n) : (float)n;
        const float2 p = tp[la], q = tq[la];
        gacc = fmaf(f, q.y * p.x - q.x * p.y, gacc);  // Re(conj(q) i f p)
      }
    } else {
      int li = 1, lj = 1;
      for (int k = 0; k < g.ki; ++k) li *= D;
      for (int k = 0; k < g.kj; ++k) lj *= D;
      const float2 *A = a.A[table_slot(g.type)];
      const int nf = nt / (D * D);
      for (int blk = wave; blk < NB; blk += kBlock / 64) {
        const int lo = blk_lo(g.kind, D, blk), b = blk_hi(g.kind, D, blk) - lo + 1;
        const float2 *Ab = A + a.boff[blk];
        for (int f = lane; f < nf; f += 64) {
          const int fb = fuse_fbase<D>(f, a.s, g.ki, g.kj);
          float2 v[D], w[D];
#pragma unroll
          for (int p = 0; p < D; ++p)
            if (p < b) {
              const int ix = fb + (lo + p) * li + blk_nj(g.kind, D, blk, lo + p) * lj;
              v[p] = tp[ix];
              w[p] = tq[ix];
            }
#pragma unroll
          for (int p = 0; p < D; ++p)
            if (p < b) {
              float2 acc = make_float2(0.f, 0.f);
#pragma unroll
              for (int q = 0; q < D; ++q)
                if (q < b) {
                  const float2 tt = cmul(Ab[p * b + q], v[q], false);
                  acc.x += tt.x;
                  acc.y += tt.y;
                }
              gacc = fmaf(w[p].x, acc.x, fmaf(w[p].y, acc.y, gacc));  // Re(conj(lam) acc)
            }
        }
      }
    }
    const double sg = block_sum_d((double)gacc, red);  // its barriers also order the reads above
    if (threadIdx.x == 0) partial[(size_t)g.k * rs + t] = sg;
    // phi <- U^+ phi, lam <- U^+ lam
    if (g.kj < 0) {
      fuse_diag<D>(tp, g, nt, U, true);
      fuse_diag<D>(tq, g, nt, U, true);
    } else {
      fuse_pair<D>(tp, g, a, nt, U, true);
      fuse_pair<D>(tq, g, a, nt, U, true);
    }
    __syncthreads();
  }
  fuse_store<D>(tp, phi, a, base, nt);
  fuse_store<D>(tq, lam, a, base, nt);
}

#define FUSE_D_SWITCH(d, STMT)                                                                 \
  switch (d) {                                                                                 \
    case 2: { constexpr int D = 2; STMT; } break;                                              \
    case 4: { constexpr int D = 4; STMT; } break;                                              \
    case 6: { constexpr int D = 6; STMT; } break;                                              \
    case 8: { constexpr int D = 8; STMT; } break;                                              \
    default: return set_error(FOCK_ERR_UNSUPPORTED, "gate fusion needs d in {2, 4, 6, 8}, got %d", d); \
  }

int launch_fuse_fwd(int d, const FuseArgs &a, const float2 *src, float2 *dst, const float2 *utab, hipStream_t s) {
  FUSE_D_SWITCH(d, hipLaunchKernelGGL(k_fuse_fwd<D>, dim3(a.ntile), dim3(kBlock), 0, s, a, src, dst, utab));
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_fuse_adj(int d, const FuseArgs &a, float2 *phi, float2 *lam, const float2 *utab, double *partial, int rs,
                    hipStream_t s) {
  FUSE_D_SWITCH(d, hipLaunchKernelGGL(k_fuse_adj<D>, dim3(a.ntile), dim3(kBlock), 0, s, a, phi, lam, utab, partial,
                                      rs));
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
