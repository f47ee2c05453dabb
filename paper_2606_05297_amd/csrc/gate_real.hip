// Real states, d = 8: the gates of the real generators HR = a_i^+ a_j - h.c.
// and PR = a_i a_j - h.c. (Sec. II.B) and their reverse steps on float32
// amplitudes.
//
// H (Sec. III) has real matrix elements in the Fock basis, and HR and PR are
// real antisymmetric, so exp(theta A) is a real orthogonal matrix.  A real
// psi0 therefore stays real through every gate of such a circuit, and so do
// H psi and the reverse sweep's phi and lambda; a state needs 4 bytes per
// amplitude instead of 8.  The gate tables are the complex ones (their
// imaginary parts are rounding noise around zero), read through their real
// parts.  Work decomposition and memory order are those of the complex
// kernels: one lane per fiber and one wave per group of conserved blocks for
// pairs (i, j) with i >= 1, 64-fiber LDS tiles walked four per workgroup for
// the pairs (0, j), and the parity-selected blocks for the top pair of the
// parity-halved layout.
#include "gate_real_groups.h"

namespace fock {

using namespace rgates;

namespace {

// ---------------------------------------------------------------- pairs (i, j), i >= 1
// One lane per fiber, 64 consecutive fibers per workgroup, wave = block group.
template <int KIND, bool DAG>
__global__ __launch_bounds__(kBlock) void k_rgate2(const float *src, float *psi, const float2 *__restrict__ U,
                                                   GateLaunch g) {
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t f = (uint32_t)vb * 64 + lane;
  if (f >= g.nfib) return;
  const uint32_t fb = fiber_base(f, g, kRD);
  const float *sb = src + fb;
  float *base = psi + fb;
  switch (wave) {
    case 0: rgate_group<KIND, DAG, 0, false>(sb, base, g.si, g.sj, U, 0); break;
    case 1: rgate_group<KIND, DAG, 1, false>(sb, base, g.si, g.sj, U, 0); break;
    case 2: rgate_group<KIND, DAG, 2, false>(sb, base, g.si, g.sj, U, 0); break;
    default: rgate_group<KIND, DAG, 3, false>(sb, base, g.si, g.sj, U, 0); break;
  }
}

template <int KIND, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_rgate2_adj(float *__restrict__ phi, float *__restrict__ lam,
                                                       const float2 *__restrict__ U, const float2 *__restrict__ A,
                                                       double *__restrict__ partial, GateLaunch g) {
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t f = (uint32_t)vb * 64 + lane;
  float gacc = 0.f;
  if (f < g.nfib) {
    const uint32_t fb = fiber_base(f, g, kRD);
    float *pb = phi + fb, *lb = lam + fb;
    switch (wave) {
      case 0: gacc = radj_group<KIND, 0, WPHI, false>(pb, lb, g.si, g.sj, U, A, 0); break;
      case 1: gacc = radj_group<KIND, 1, WPHI, false>(pb, lb, g.si, g.sj, U, A, 0); break;
      case 2: gacc = radj_group<KIND, 2, WPHI, false>(pb, lb, g.si, g.sj, U, A, 0); break;
      default: gacc = radj_group<KIND, 3, WPHI, false>(pb, lb, g.si, g.sj, U, A, 0); break;
    }
  }
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

// ---------------------------------------------------------------- the top pair of the parity-halved layout
// A workgroup takes 128 consecutive lower indices f in two passes, one per
// value P of the lower modes' parity plus the sector: in pass P lane l takes
// the one of f0 + 2l, f0 + 2l + 1 (they differ in n_0 by one, so in parity)
// whose parity is P.  The parity is then uniform and known at compile time in
// each pass, so only the stored blocks are loaded and computed; a pass's
// member loads cover every other float of a 512-byte run, the other pass the
// rest.
constexpr int kRHalfPer = 128;

__device__ __forceinline__ uint32_t rhalf_f(uint32_t f0, int lane, int P, int sector) {
  const uint32_t fe = f0 + 2u * (uint32_t)lane;
  return fe + (uint32_t)(((octal_digit_parity(fe) + sector) & 1) != P);
}

template <int KIND, bool DAG, int P>
__device__ __forceinline__ void rhalf_pass(const float *src, float *psi, const float2 *__restrict__ U,
                                           const GateLaunch &g, int sector, uint32_t f0, int wave, int lane) {
  const uint32_t f = rhalf_f(f0, lane, P, sector);
  if (f >= g.nfib) return;
  switch (wave) {
    case 0: rgate_group<KIND, DAG, 0, true, const float2 *__restrict__, P>(src + f, psi + f, g.si, g.sj, U, P); break;
    case 1: rgate_group<KIND, DAG, 1, true, const float2 *__restrict__, P>(src + f, psi + f, g.si, g.sj, U, P); break;
    case 2: rgate_group<KIND, DAG, 2, true, const float2 *__restrict__, P>(src + f, psi + f, g.si, g.sj, U, P); break;
    default: rgate_group<KIND, DAG, 3, true, const float2 *__restrict__, P>(src + f, psi + f, g.si, g.sj, U, P); break;
  }
}

template <int KIND, bool DAG>
__global__ __launch_bounds__(kBlock) void k_rgate2_half(const float *src, float *psi, const float2 *__restrict__ U,
                                                        GateLaunch g, int sector) {
  const uint32_t f0 = (uint32_t)xcd_remap(blockIdx.x, gridDim.x) * kRHalfPer;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  rhalf_pass<KIND, DAG, 0>(src, psi, U, g, sector, f0, wave, lane);
  rhalf_pass<KIND, DAG, 1>(src, psi, U, g, sector, f0, wave, lane);
}

template <int KIND, bool WPHI, int P>
__device__ __forceinline__ float rhalf_adj_pass(float *phi, float *lam, const float2 *__restrict__ U,
                                                const float2 *__restrict__ A, const GateLaunch &g, int sector,
                                                uint32_t f0, int wave, int lane) {
  const uint32_t f = rhalf_f(f0, lane, P, sector);
  if (f >= g.nfib) return 0.f;
  using CP = const float2 *__restrict__;
  switch (wave) {
    case 0: return radj_group<KIND, 0, WPHI, true, CP, P>(phi + f, lam + f, g.si, g.sj, U, A, P);
    case 1: return radj_group<KIND, 1, WPHI, true, CP, P>(phi + f, lam + f, g.si, g.sj, U, A, P);
    case 2: return radj_group<KIND, 2, WPHI, true, CP, P>(phi + f, lam + f, g.si, g.sj, U, A, P);
    default: return radj_group<KIND, 3, WPHI, true, CP, P>(phi + f, lam + f, g.si, g.sj, U, A, P);
  }
}

template <int KIND, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_rgate2_adj_half(float *__restrict__ phi, float *__restrict__ lam,
                                                            const float2 *__restrict__ U,
                                                            const float2 *__restrict__ A, double *__restrict__ partial,
                                                            GateLaunch g, int sector) {
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t f0 = (uint32_t)vb * kRHalfPer;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float gacc = rhalf_adj_pass<KIND, WPHI, 0>(phi, lam, U, A, g, sector, f0, wave, lane);
  gacc += rhalf_adj_pass<KIND, WPHI, 1>(phi, lam, U, A, g, sector, f0, wave, lane);
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

// ---------------------------------------------------------------- pairs (0, j): pipelined LDS tiles
// A tile is 64 fibers of 64 members (n_0 = a, n_j = b at b * 8 + a, rows padded
// to 65 floats); a thread moves 4 float4 (4 consecutive n_0 values each) per
// tile.  A workgroup walks kRTiles tiles; the next tile's loads are issued
// before the current tile is computed and stored.
constexpr int kRFL = 64, kRST = kRD * kRD + 1, kRPer = kRFL * kRD * kRD / 4 / kBlock;
// Tiles per workgroup: two (1024 workgroups at L = 8 parity-halved) measured
// 4-5% faster per ADAPT step than one or four.
constexpr int kRTiles = 2;

__device__ __forceinline__ void rm0_bases(uint32_t tile, const GateLaunch &g, uint32_t *fb) {
  if (threadIdx.x < kRFL) fb[threadIdx.x] = fiber_base(tile * kRFL + threadIdx.x, g, kRD);
}

__device__ __forceinline__ void rm0_coord(int i, int &fl, int &b, int &a) {
  constexpr int PERB = kRFL * kRD / 4;  // float4 per row b of a tile
  const int e = threadIdx.x + i * kBlock, r = e % PERB;
  b = e / PERB;
  fl = r / (kRD / 4);
  a = 4 * (r % (kRD / 4));
}

__device__ __forceinline__ void rm0_gload(const float *src, const uint32_t *fb, uint32_t sj, float4 (&buf)[kRPer]) {
#pragma unroll
  for (int i = 0; i < kRPer; ++i) {
    int fl, b, a;
    rm0_coord(i, fl, b, a);
    buf[i] = *reinterpret_cast<const float4 *>(src + fb[fl] + (uint32_t)a + (uint32_t)b * sj);
  }
}

__device__ __forceinline__ void rm0_lds_put(float *tile, const float4 (&buf)[kRPer]) {
#pragma unroll
  for (int i = 0; i < kRPer; ++i) {
    int fl, b, a;
    rm0_coord(i, fl, b, a);
    float *tp = tile + fl * kRST + b * kRD + a;
    tp[0] = buf[i].x;
    tp[1] = buf[i].y;
    tp[2] = buf[i].z;
    tp[3] = buf[i].w;
  }
}

__device__ __forceinline__ void rm0_gstore(float *dst, const uint32_t *fb, uint32_t sj, const float *tile) {
#pragma unroll
  for (int i = 0; i < kRPer; ++i) {
    int fl, b, a;
    rm0_coord(i, fl, b, a);
    const float *tp = tile + fl * kRST + b * kRD + a;
    *reinterpret_cast<float4 *>(dst + fb[fl] + (uint32_t)a + (uint32_t)b * sj) =
        make_float4(tp[0], tp[1], tp[2], tp[3]);
  }
}

template <int KIND, bool DAG>
__global__ __launch_bounds__(kBlock) void k_rgate2_m0p(const float *src, float *psi, const float2 *__restrict__ U,
                                                       GateLaunch g) {
  __shared__ float tile[kRFL * kRST];
  __shared__ uint32_t fbase[2][kRFL];
  const uint32_t t0 = (uint32_t)xcd_remap(blockIdx.x, gridDim.x) * kRTiles;
  float4 buf[kRPer];
  rm0_bases(t0, g, fbase[0]);
  rm0_bases(t0 + 1, g, fbase[1]);
  __syncthreads();
  rm0_gload(src, fbase[0], g.sj, buf);
  rm0_lds_put(tile, buf);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll 1
  for (int t = 0; t < kRTiles; ++t) {
    const bool more = t + 1 < kRTiles;
    if (more) rm0_gload(src, fbase[(t + 1) & 1], g.sj, buf);
    float *base = tile + lane * kRST;
    switch (wave) {
      case 0: rgate_group<KIND, DAG, 0, false>(base, base, 1u, (uint32_t)kRD, U, 0); break;
      case 1: rgate_group<KIND, DAG, 1, false>(base, base, 1u, (uint32_t)kRD, U, 0); break;
      case 2: rgate_group<KIND, DAG, 2, false>(base, base, 1u, (uint32_t)kRD, U, 0); break;
      default: rgate_group<KIND, DAG, 3, false>(base, base, 1u, (uint32_t)kRD, U, 0); break;
    }
    __syncthreads();
    rm0_gstore(psi, fbase[t & 1], g.sj, tile);
    __syncthreads();
    if (more) {
      rm0_lds_put(tile, buf);
      if (t + 2 < kRTiles) rm0_bases(t0 + t + 2, g, fbase[t & 1]);
      __syncthreads();
    }
  }
}

template <int KIND, bool WPHI>
__global__ __launch_bounds__(kBlock) void k_rgate2_adj_m0p(float *__restrict__ phi, float *__restrict__ lam,
                                                           const float2 *__restrict__ U, const float2 *__restrict__ A,
                                                           double *__restrict__ partial, GateLaunch g) {
  __shared__ float tp[kRFL * kRST], tl[kRFL * kRST];
  __shared__ uint32_t fbase[2][kRFL];
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t t0 = (uint32_t)vb * kRTiles;
  float4 bp[kRPer], bl[kRPer];
  rm0_bases(t0, g, fbase[0]);
  rm0_bases(t0 + 1, g, fbase[1]);
  __syncthreads();
  rm0_gload(phi, fbase[0], g.sj, bp);
  rm0_gload(lam, fbase[0], g.sj, bl);
  rm0_lds_put(tp, bp);
  rm0_lds_put(tl, bl);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float gacc = 0.f;
#pragma unroll 1
  for (int t = 0; t < kRTiles; ++t) {
    const bool more = t + 1 < kRTiles;
    if (more) {
      rm0_gload(phi, fbase[(t + 1) & 1], g.sj, bp);
      rm0_gload(lam, fbase[(t + 1) & 1], g.sj, bl);
    }
    float *pb = tp + lane * kRST, *lb = tl + lane * kRST;
    switch (wave) {
      case 0: gacc += radj_group<KIND, 0, WPHI, false>(pb, lb, 1u, (uint32_t)kRD, U, A, 0); break;
      case 1: gacc += radj_group<KIND, 1, WPHI, false>(pb, lb, 1u, (uint32_t)kRD, U, A, 0); break;
      case 2: gacc += radj_group<KIND, 2, WPHI, false>(pb, lb, 1u, (uint32_t)kRD, U, A, 0); break;
      default: gacc += radj_group<KIND, 3, WPHI, false>(pb, lb, 1u, (uint32_t)kRD, U, A, 0); break;
    }
    __syncthreads();
    if (WPHI) rm0_gstore(phi, fbase[t & 1], g.sj, tp);
    rm0_gstore(lam, fbase[t & 1], g.sj, tl);
    __syncthreads();
    if (more) {
      rm0_lds_put(tp, bp);
      rm0_lds_put(tl, bl);
      if (t + 2 < kRTiles) rm0_bases(t0 + t + 2, g, fbase[t & 1]);
      __syncthreads();
    }
  }
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

// ---------------------------------------------------------------- real <-> complex
__global__ __launch_bounds__(kBlock) void k_real_to_complex(const float4 *__restrict__ r, float4 *__restrict__ c,
                                                            uint32_t n4) {
  const uint32_t i = (uint32_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n4) return;
  const float4 v = r[i];
  c[2 * i] = make_float4(v.x, 0.f, v.y, 0.f);
  c[2 * i + 1] = make_float4(v.z, 0.f, v.w, 0.f);
}

__global__ __launch_bounds__(kBlock) void k_complex_to_real(const float4 *__restrict__ c, float4 *__restrict__ r,
                                                            uint32_t n4) {
  const uint32_t i = (uint32_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n4) return;
  const float4 a = c[2 * i], b = c[2 * i + 1];
  r[i] = make_float4(a.x, a.z, b.x, b.z);
}

// Largest |Im| of a complex state, as a per-workgroup max of the bit patterns
// of |Im| (non-negative floats order like their bits); zero iff every
// imaginary part is +-0.
__global__ __launch_bounds__(kBlock) void k_imag_any(const float2 *__restrict__ c, uint32_t n,
                                                     unsigned int *__restrict__ flag) {
  const uint32_t i = (uint32_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned int bits = 0u;
  if (i < n) bits = __float_as_uint(fabsf(c[i].y));
  // wave-level max, then one atomic per wave on a device word
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bits = max(bits, (unsigned int)__shfl_xor((int)bits, o, 64));
  if ((threadIdx.x & 63) == 0 && bits) atomicMax(flag, bits);
}

struct RealSel {
  bool ok;
  bool m0p;
  bool half_top;
};

RealSel real_select(const Geometry &g, int i, int j) {
  RealSel r{false, false, false};
  if (g.d != kRD || g.L < 3) return r;
  if (g.half && j == g.L - 1) {
    r.ok = i == g.L - 2;
    r.half_top = true;
    return r;
  }
  if (i == 0) {
    const uint32_t nfib = g.n_amp / (uint32_t)(kRD * kRD);
    r.ok = nfib % (uint32_t)(kRFL * kRTiles) == 0;
    r.m0p = true;
    return r;
  }
  r.ok = true;
  return r;
}

GateLaunch rlaunch(const Geometry &g, int i, int j, bool half_top) {
  GateLaunch gl = gate_launch_params(g, i, j);
  if (half_top) {
    gl.nfib = gl.si;  // d^(L-2) lower indices, 32 stored members each
  }
  return gl;
}

}  // namespace

bool real_gate_supported(const Geometry &g, int i, int j) { return real_select(g, i, j).ok; }

int real_gate_blocks(const Geometry &g, int i, int j) {
  const RealSel r = real_select(g, i, j);
  const GateLaunch gl = rlaunch(g, i, j, r.half_top);
  const uint32_t per = r.m0p ? (uint32_t)(kRFL * kRTiles) : (r.half_top ? (uint32_t)kRHalfPer : 64u);
  return (int)((gl.nfib + per - 1) / per);
}

template <int K, bool DG>
static void rg_launch(const RealSel &r, int G, hipStream_t s, const float *src, float *psi, const float2 *U,
                      const GateLaunch &gl, int sector) {
  if (r.m0p) hipLaunchKernelGGL((k_rgate2_m0p<K, DG>), dim3(G), dim3(kBlock), 0, s, src, psi, U, gl);
  else if (r.half_top) hipLaunchKernelGGL((k_rgate2_half<K, DG>), dim3(G), dim3(kBlock), 0, s, src, psi, U, gl, sector);
  else hipLaunchKernelGGL((k_rgate2<K, DG>), dim3(G), dim3(kBlock), 0, s, src, psi, U, gl);
}

template <int K, bool W>
static void ra_launch(const RealSel &r, int G, hipStream_t s, float *phi, float *lam, const float2 *U,
                      const float2 *A, double *partial, const GateLaunch &gl, int sector) {
  if (r.m0p)
    hipLaunchKernelGGL((k_rgate2_adj_m0p<K, W>), dim3(G), dim3(kBlock), 0, s, phi, lam, U, A, partial, gl);
  else if (r.half_top)
    hipLaunchKernelGGL((k_rgate2_adj_half<K, W>), dim3(G), dim3(kBlock), 0, s, phi, lam, U, A, partial, gl, sector);
  else
    hipLaunchKernelGGL((k_rgate2_adj<K, W>), dim3(G), dim3(kBlock), 0, s, phi, lam, U, A, partial, gl);
}

int launch_rgate(const Geometry &g, int i, int j, int kind, bool dag, const float2 *U, const float *src, float *psi,
                 hipStream_t s) {
  const RealSel r = real_select(g, i, j);
  if (!r.ok) return set_error(FOCK_ERR_UNSUPPORTED, "real-state gate on (%d,%d) at L=%d, d=%d", i, j, g.L, g.d);
  const GateLaunch gl = rlaunch(g, i, j, r.half_top);
  const int G = real_gate_blocks(g, i, j);
  if (kind == KIND_SUM) {
    if (dag) rg_launch<KIND_SUM, true>(r, G, s, src, psi, U, gl, g.sector);
    else rg_launch<KIND_SUM, false>(r, G, s, src, psi, U, gl, g.sector);
  } else {
    if (dag) rg_launch<KIND_DIFF, true>(r, G, s, src, psi, U, gl, g.sector);
    else rg_launch<KIND_DIFF, false>(r, G, s, src, psi, U, gl, g.sector);
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_rgate_adj(const Geometry &g, int i, int j, int kind, const float2 *U, const float2 *A, float *phi,
                     float *lam, double *partial, hipStream_t s, bool write_phi) {
  const RealSel r = real_select(g, i, j);
  if (!r.ok) return set_error(FOCK_ERR_UNSUPPORTED, "real-state reverse step on (%d,%d)", i, j);
  const GateLaunch gl = rlaunch(g, i, j, r.half_top);
  const int G = real_gate_blocks(g, i, j);
  if (kind == KIND_SUM) {
    if (write_phi) ra_launch<KIND_SUM, true>(r, G, s, phi, lam, U, A, partial, gl, g.sector);
    else ra_launch<KIND_SUM, false>(r, G, s, phi, lam, U, A, partial, gl, g.sector);
  } else {
    if (write_phi) ra_launch<KIND_DIFF, true>(r, G, s, phi, lam, U, A, partial, gl, g.sector);
    else ra_launch<KIND_DIFF, false>(r, G, s, phi, lam, U, A, partial, gl, g.sector);
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_real_convert(uint32_t n, bool to_complex, const void *src, void *dst, hipStream_t s) {
  if (n % 4) return set_error(FOCK_ERR_SIZE, "real/complex conversion of %u amplitudes (multiple of 4 needed)", n);
  const uint32_t n4 = n / 4;
  const int G = (int)((n4 + kBlock - 1) / kBlock);
  if (to_complex)
    hipLaunchKernelGGL(k_real_to_complex, dim3(G), dim3(kBlock), 0, s, (const float4 *)src, (float4 *)dst, n4);
  else
    hipLaunchKernelGGL(k_complex_to_real, dim3(G), dim3(kBlock), 0, s, (const float4 *)src, (float4 *)dst, n4);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_imag_any(const float2 *c, uint32_t n, unsigned int *flag, hipStream_t s) {
  const int G = (int)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_imag_any, dim3(G), dim3(kBlock), 0, s, c, n, flag);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
