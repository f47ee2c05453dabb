// Single-mode squeezer gates (Sec. II.B): the generators SR = (a^2 - a^+2)/2
// and SI = i (a^2 + a^+2)/2 connect n and n +- 2 on one mode r, so a gate is a
// dense d x d unitary on each fibre (the d amplitudes along mode r for fixed
// other digits), zero between levels of opposite parity.
//
// Work decomposition: one thread per fibre.  Fibre f has base
// (f / s) * s * d + f % s and members base + m s, s = d^r: consecutive threads
// take consecutive fibres, so each member load of a wavefront is one
// contiguous run (mode 0: each thread owns one contiguous row).  U and A are
// wavefront-uniform d x d tables (scalar loads); the kernels are HBM-bound at
// 16 B (forward, pool scoring) or 32 B (reverse step) per amplitude.
#include "device_common.h"

namespace fock {

struct Gate1Launch {
  uint32_t nfib;  // d^(L-1)
  uint32_t s;     // d^r: stride of mode r in amplitudes
};

template <int D>
__device__ __forceinline__ uint32_t fibre_base1(uint32_t f, const Gate1Launch &g) {
  return (f / g.s) * g.s * D + f % g.s;
}

// y = M x (DAG: M^+ x) for a d x d matrix with zero entries between levels of
// opposite parity.
template <int D, bool DAG>
__device__ __forceinline__ void matvec1(const float2 *__restrict__ M, const float2 (&x)[D], float2 (&y)[D]) {
#pragma unroll
  for (int p = 0; p < D; ++p) {
    float yr = 0.f, yi = 0.f;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      if ((p + q) & 1) continue;
      const float2 m = DAG ? M[q * D + p] : M[p * D + q];
      const float mi = DAG ? -m.y : m.y;
      yr = fmaf(m.x, x[q].x, fmaf(-mi, x[q].y, yr));
      yi = fmaf(m.x, x[q].y, fmaf(mi, x[q].x, yi));
    }
    y[p] = make_float2(yr, yi);
  }
}

template <int D>
__device__ __forceinline__ void load1(const float2 *__restrict__ p, uint32_t s, float2 (&x)[D]) {
#pragma unroll
  for (int m = 0; m < D; ++m) x[m] = p[(size_t)m * s];
}

template <int D>
__device__ __forceinline__ void store1(float2 *__restrict__ p, uint32_t s, const float2 (&x)[D]) {
#pragma unroll
  for (int m = 0; m < D; ++m) p[(size_t)m * s] = x[m];
}

// psi <- U src (DAG: U^+ src); src may equal psi.
template <int D, bool DAG>
__global__ __launch_bounds__(kBlock) void k_gate1(const float2 *src, float2 *psi, const float2 *__restrict__ U,
                                                  Gate1Launch g) {
  const uint32_t f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= g.nfib) return;
  const uint32_t b = fibre_base1<D>(f, g);
  float2 x[D], y[D];
  load1<D>(src + b, g.s, x);
  matvec1<D, DAG>(U, x, y);
  store1<D>(psi + b, g.s, y);
}

// Reverse step of one squeezer gate: this workgroup's share of
// Re<lam|A phi>, then phi <- U^+ phi and lam <- U^+ lam.
template <int D>
__global__ __launch_bounds__(kBlock) void k_gate1_adj(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                      const float2 *__restrict__ U, const float2 *__restrict__ A,
                                                      double *__restrict__ partial, Gate1Launch g) {
  __shared__ double red[4];
  const uint32_t f = blockIdx.x * kBlock + threadIdx.x;
  float gacc = 0.f;
  if (f < g.nfib) {
    const uint32_t b = fibre_base1<D>(f, g);
    float2 x[D], l[D], ax[D];
    load1<D>(phi + b, g.s, x);
    load1<D>(lam + b, g.s, l);
    matvec1<D, false>(A, x, ax);
#pragma unroll
    for (int p = 0; p < D; ++p) gacc = fmaf(l[p].x, ax[p].x, fmaf(l[p].y, ax[p].y, gacc));
    float2 y[D];
    matvec1<D, true>(U, x, y);
    store1<D>(phi + b, g.s, y);
    matvec1<D, true>(U, l, y);
    store1<D>(lam + b, g.s, y);
  }
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = sg;
}

// Pool scoring of one squeezer entry: this workgroup's share of
// 2 Re<hpsi|A psi>.
template <int D>
__global__ __launch_bounds__(kBlock) void k_pool1(const float2 *__restrict__ psi, const float2 *__restrict__ hpsi,
                                                  const float2 *__restrict__ A, double *__restrict__ partial,
                                                  Gate1Launch g) {
  __shared__ double red[4];
  const uint32_t f = blockIdx.x * kBlock + threadIdx.x;
  float v = 0.f;
  if (f < g.nfib) {
    const uint32_t b = fibre_base1<D>(f, g);
    float2 x[D], h[D], ax[D];
    load1<D>(psi + b, g.s, x);
    load1<D>(hpsi + b, g.s, h);
    matvec1<D, false>(A, x, ax);
#pragma unroll
    for (int p = 0; p < D; ++p) v = fmaf(h[p].x, ax[p].x, fmaf(h[p].y, ax[p].y, v));
  }
  const double s = block_sum_d(2.0 * (double)v, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

static Gate1Launch make_gate1_launch(const Geometry &g, int r) {
  Gate1Launch a;
  a.nfib = g.n_amp / (uint32_t)g.d;
  uint32_t s = 1;
  for (int k = 0; k < r; ++k) s *= (uint32_t)g.d;
  a.s = s;
  return a;
}

static int gate1_grid(const Gate1Launch &a) { return (int)((a.nfib + kBlock - 1) / kBlock); }

#define G1_D_SWITCH(d, STMT)                                                                          \
  switch (d) {                                                                                        \
    case 2: { constexpr int D = 2; STMT; } break;                                                     \
    case 3: { constexpr int D = 3; STMT; } break;                                                     \
    case 4: { constexpr int D = 4; STMT; } break;                                                     \
    case 5: { constexpr int D = 5; STMT; } break;                                                     \
    case 6: { constexpr int D = 6; STMT; } break;                                                     \
    case 7: { constexpr int D = 7; STMT; } break;                                                     \
    case 8: { constexpr int D = 8; STMT; } break;                                                     \
    case 9: { constexpr int D = 9; STMT; } break;                                                     \
    case 10: { constexpr int D = 10; STMT; } break;                                                   \
    case 11: { constexpr int D = 11; STMT; } break;                                                   \
    case 12: { constexpr int D = 12; STMT; } break;                                                   \
    case 13: { constexpr int D = 13; STMT; } break;                                                   \
    case 14: { constexpr int D = 14; STMT; } break;                                                   \
    case 15: { constexpr int D = 15; STMT; } break;                                                   \
    case 16: { constexpr int D = 16; STMT; } break;                                                   \
    default: return set_error(FOCK_ERR_UNSUPPORTED, "squeezer gate: d=%d unsupported", d);           \
  }

int launch_gate1(const Geometry &g, int r, bool dag, const float2 *U, const float2 *src, float2 *psi,
                 hipStream_t s) {
  if (g.half) return set_error(FOCK_ERR_UNSUPPORTED, "squeezers in the parity-halved layout");
  const Gate1Launch a = make_gate1_launch(g, r);
  const dim3 grid(gate1_grid(a));
  if (dag) G1_D_SWITCH(g.d, hipLaunchKernelGGL((k_gate1<D, true>), grid, dim3(kBlock), 0, s, src, psi, U, a))
  else G1_D_SWITCH(g.d, hipLaunchKernelGGL((k_gate1<D, false>), grid, dim3(kBlock), 0, s, src, psi, U, a))
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_gate1_adj(const Geometry &g, int r, const float2 *U, const float2 *A, float2 *phi, float2 *lam,
                     double *partial, hipStream_t s) {
  if (g.half) return set_error(FOCK_ERR_UNSUPPORTED, "squeezers in the parity-halved layout");
  const Gate1Launch a = make_gate1_launch(g, r);
  const dim3 grid(gate1_grid(a));
  G1_D_SWITCH(g.d, hipLaunchKernelGGL(k_gate1_adj<D>, grid, dim3(kBlock), 0, s, phi, lam, U, A, partial, a))
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_pool1(const Geometry &g, int r, const float2 *A, const float2 *psi, const float2 *hpsi, double *partial,
                 int *nblocks, hipStream_t s) {
  if (g.half) return set_error(FOCK_ERR_UNSUPPORTED, "squeezers in the parity-halved layout");
  const Gate1Launch a = make_gate1_launch(g, r);
  *nblocks = gate1_grid(a);
  const dim3 grid(*nblocks);
  G1_D_SWITCH(g.d, hipLaunchKernelGGL(k_pool1<D>, grid, dim3(kBlock), 0, s, psi, hpsi, A, partial, a))
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
