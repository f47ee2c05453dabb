// Runs of real gates (HR, PR; d = 8, float32 amplitudes) as one pass over the
// state.
//
// Consecutive gates of a circuit whose pairs lie inside three consecutive
// modes (a, a+1, a+2) only mix amplitudes that agree on every other mode: for
// fixed digits of the other modes, the 512 amplitudes over (n_a, n_{a+1},
// n_{a+2}) are mapped among themselves.  A workgroup stages R such 512-sets
// (R "rests") in LDS, applies the run's gates there one after another with the
// per-fiber block arithmetic of the single-gate kernels (Sec. II.B), and writes
// the tile back, so the state is read and written once per run instead of once
// per gate, with the same results bit for bit.  The reverse form stages phi and
// lambda and takes the run's reverse steps in reverse gate order (Sec. IV.B
// gradient identity), each writing its tile's share of lambda . A_k phi.
//
// Rests of a tile: R consecutive values of the modes below a when d^a >= R
// (tile kind 2, a >= 2); else all d^a values of the modes below a times R / d^a
// consecutive values of the modes above a+2 (kind 0: a = 0, kind 1: a = 1).
// Either way the tile is read and written in contiguous runs of >= R floats.
// The modes above a+2 may include the top mode of the parity-halved layout (its
// stored index m): the gates of a run keep the parity of modes a..a+2, so the
// stored positions of a tile are those of the full layout with m as the digit.
//
// LDS layout of a tile (lo: rest digits below a, hl: rest digits above a+2,
// x, y, z: n_a, n_{a+1}, n_{a+2}):  lo + SH hl + RLO (x + 8 y) + SZ z.  A gate
// on tile modes (o, o+1) has fibers (rest, third digit w); a wave takes one
// conserved-block group for 64 fibers at a time, lanes over the rests first.
// SZ and SH are padded so that the 32 lanes of each half-wave hit 32 distinct
// banks in every gate phase.
#include <cstring>

#include "gate_real_groups.h"

namespace fock {

using namespace rgates;

namespace {

constexpr int kRFuseR = 32;     // rests per forward tile (64 KiB of LDS)
constexpr int kRFuseRAdj = 16;  // rests per reverse tile (phi and lambda: 2 x 32 KiB)

template <int TK, int R>
struct RTile {
  static_assert(R == 16 || R == 32, "tile of 16 or 32 rests");
  static constexpr int RLO = TK == 0 ? 1 : (TK == 1 ? 8 : R);
  static constexpr int RHI = R / RLO;
  static constexpr int SZ = TK == 0 ? 65 : (TK == 1 ? (R == 32 ? 512 : 520) : (R == 32 ? 2048 : 1040));
  static constexpr int SH = TK == 0 ? (R == 32 ? 521 : 546) : (TK == 1 ? (R == 32 ? 4104 : 4176) : 0);
  static constexpr int SIZE = SH * (RHI - 1) + SZ * 7 + RLO * 64;
  static constexpr int PER = R * 512 / 4 / kBlock;  // float4 per thread per tile
  // float4 writes into LDS need 16-byte aligned rows (kind 0 writes floats)
  static_assert(TK == 0 || (SZ % 4 == 0 && SH % 4 == 0), "aligned tile rows");
};

struct RFuseArgs {
  uint32_t sa;        // d^a: stride of n_a
  uint32_t lo_tiles;  // kind 2: tiles per value of the modes above a+2 (d^a / R)
  int ng;
  int kind[kRFuseMax], o[kRFuseMax];
  const float2 *U[kRFuseMax];
  const float2 *A[kRFuseMax];
  double *part[kRFuseMax];
};

template <int TK, int R>
__device__ __forceinline__ uint32_t rf_tile_base(uint32_t t, const RFuseArgs &a) {
  if (TK < 2) return t * (uint32_t)(R * 512);
  const uint32_t hi = t / a.lo_tiles;
  return hi * a.sa * 512u + (t - hi * a.lo_tiles) * (uint32_t)R;
}

// float4 chunk c of a tile: global offset from the tile base and LDS offset.
template <int TK, int R>
__device__ __forceinline__ void rf_coord(int c, uint32_t sa, uint32_t &go, int &lo) {
  using T = RTile<TK, R>;
  const int e = 4 * c;
  if (TK == 0) {  // e = x + 8 y + 64 z + 512 hl, contiguous
    go = (uint32_t)e;
    lo = (e & 63) + T::SZ * ((e >> 6) & 7) + T::SH * (e >> 9);
  } else if (TK == 1) {  // e = lo + 8 (x + 8 y + 64 z) + 4096 hl, contiguous
    go = (uint32_t)e;
    lo = (e & 511) + T::SZ * ((e >> 9) & 7) + T::SH * (e >> 12);
  } else {  // e = lo + R (x + 8 y + 64 z)
    const int l = e % R, xyz = e / R;
    go = (uint32_t)l + sa * (uint32_t)xyz;
    lo = l + R * (xyz & 63) + T::SZ * (xyz >> 6);
  }
}

template <int TK>
__device__ __forceinline__ void rf_put(float *p, float4 v) {
  if (TK == 0) {
    p[0] = v.x;
    p[1] = v.y;
    p[2] = v.z;
    p[3] = v.w;
  } else {
    *reinterpret_cast<float4 *>(p) = v;
  }
}

template <int TK>
__device__ __forceinline__ float4 rf_get(const float *p) {
  if (TK == 0) return make_float4(p[0], p[1], p[2], p[3]);
  return *reinterpret_cast<const float4 *>(p);
}

template <int TK, int R>
__device__ __forceinline__ void rf_gload(const float *__restrict__ src, uint32_t sa, float4 (&v)[RTile<TK, R>::PER]) {
#pragma unroll
  for (int i = 0; i < RTile<TK, R>::PER; ++i) {
    uint32_t go;
    int lo;
    rf_coord<TK, R>(threadIdx.x + i * kBlock, sa, go, lo);
    v[i] = *reinterpret_cast<const float4 *>(src + go);
  }
}

template <int TK, int R>
__device__ __forceinline__ void rf_lput(float *tile, uint32_t sa, const float4 (&v)[RTile<TK, R>::PER]) {
#pragma unroll
  for (int i = 0; i < RTile<TK, R>::PER; ++i) {
    uint32_t go;
    int lo;
    rf_coord<TK, R>(threadIdx.x + i * kBlock, sa, go, lo);
    rf_put<TK>(tile + lo, v[i]);
  }
}

template <int TK, int R>
__device__ __forceinline__ void rf_gstore(float *__restrict__ dst, uint32_t sa, const float *tile) {
#pragma unroll
  for (int i = 0; i < RTile<TK, R>::PER; ++i) {
    uint32_t go;
    int lo;
    rf_coord<TK, R>(threadIdx.x + i * kBlock, sa, go, lo);
    *reinterpret_cast<float4 *>(dst + go) = rf_get<TK>(tile + lo);
  }
}

// The real parts of a gate's packed tables (U, and A for the reverse step)
// staged in LDS: the next gate's tables are loaded while the current gate is
// applied, so a gate phase starts without waiting on table loads.
constexpr int kTabN = 344;  // sum of b^2 over the conserved blocks at d = 8
struct LdsTab {
  const float *p;
  __device__ __forceinline__ float2 operator[](int i) const { return make_float2(p[i], 0.f); }
};
constexpr int kTabPer = (2 * kTabN + kBlock - 1) / kBlock;

// this thread's share of the tables of one gate (nt = 1: U; 2: U then A)
__device__ __forceinline__ void rf_tab_fetch(const float2 *U, const float2 *A, int nt, float (&r)[kTabPer]) {
#pragma unroll
  for (int j = 0; j < kTabPer; ++j) {
    const int e = threadIdx.x + j * kBlock;
    r[j] = e < kTabN ? U[e].x : (e < nt * kTabN ? A[e - kTabN].x : 0.f);
  }
}

__device__ __forceinline__ void rf_tab_put(float *tab, int nt, const float (&r)[kTabPer]) {
#pragma unroll
  for (int j = 0; j < kTabPer; ++j) {
    const int e = threadIdx.x + j * kBlock;
    if (e < nt * kTabN) tab[e] = r[j];
  }
}

// Fiber geometry of a gate on tile modes (O, O+1): member strides and the
// stride of the third digit w.
template <int TK, int R, int O>
struct RPhase {
  using T = RTile<TK, R>;
  static constexpr uint32_t SI = O == 0 ? T::RLO : 8 * T::RLO;
  static constexpr uint32_t SJ = O == 0 ? 8 * T::RLO : T::SZ;
  static constexpr int SW = O == 0 ? T::SZ : T::RLO;
};

template <int TK, int R>
__device__ __forceinline__ int rf_rest_off(int lane) {
  using T = RTile<TK, R>;
  const int rr = lane % R;
  return rr % T::RLO + T::SH * (rr / T::RLO);
}

// psi <- U psi on group G of every fiber of the tile (64 fibers per round).
template <int TK, int R, int KIND, int O, int G>
__device__ __forceinline__ void rf_gate(float *tile, LdsTab U, int lane) {
  using P = RPhase<TK, R, O>;
  float *rb = tile + rf_rest_off<TK, R>(lane);
#pragma unroll 1
  for (int rho = 0; rho < R / 8; ++rho) {
    float *b = rb + P::SW * (lane / R + (64 / R) * rho);
    rgate_group<KIND, false, G, false, LdsTab>(b, b, P::SI, P::SJ, U, 0);
  }
}

template <int TK, int R, int KIND, int O, int G>
__device__ __forceinline__ float rf_adj(float *tp, float *tl, LdsTab U, LdsTab A, int lane) {
  using P = RPhase<TK, R, O>;
  const int rb = rf_rest_off<TK, R>(lane);
  float g = 0.f;
#pragma unroll 1
  for (int rho = 0; rho < R / 8; ++rho) {
    const int b = rb + P::SW * (lane / R + (64 / R) * rho);
    g += radj_group<KIND, G, true, false, LdsTab>(tp + b, tl + b, P::SI, P::SJ, U, A, 0);
  }
  return g;
}

#define RF_WAVES(CALL_G)          \
  switch (wave) {                 \
    case 0: CALL_G(0); break;     \
    case 1: CALL_G(1); break;     \
    case 2: CALL_G(2); break;     \
    default: CALL_G(3); break;    \
  }

template <int TK, int R, int KIND, int O>
__device__ __forceinline__ void rf_gate_w(int wave, float *tile, LdsTab U, int lane) {
#define RFG(G) rf_gate<TK, R, KIND, O, G>(tile, U, lane)
  RF_WAVES(RFG)
#undef RFG
}

template <int TK, int R, int KIND, int O>
__device__ __forceinline__ float rf_adj_w(int wave, float *tp, float *tl, LdsTab U, LdsTab A, int lane) {
  float g = 0.f;
#define RFA(G) g = rf_adj<TK, R, KIND, O, G>(tp, tl, U, A, lane)
  RF_WAVES(RFA)
#undef RFA
  return g;
}

template <int TK>
__global__ __launch_bounds__(kBlock) void k_rfuse(const float *src, float *dst, RFuseArgs a) {
  constexpr int R = kRFuseR;
  using T = RTile<TK, R>;
  __shared__ __align__(16) float tile[T::SIZE];
  __shared__ float tab[2][kTabN];
  const uint32_t t = (uint32_t)xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t gb = rf_tile_base<TK, R>(t, a);
  float r[kTabPer];
  {
    float4 v[T::PER];
    rf_gload<TK, R>(src + gb, a.sa, v);
    rf_tab_fetch(a.U[0], nullptr, 1, r);
    rf_lput<TK, R>(tile, a.sa, v);
    rf_tab_put(tab[0], 1, r);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int gi = 0; gi < a.ng; ++gi) {
    const bool more = gi + 1 < a.ng;
    if (more) rf_tab_fetch(a.U[gi + 1], nullptr, 1, r);
    const LdsTab U{tab[gi & 1]};
    if (a.kind[gi] == KIND_SUM) {
      if (a.o[gi] == 0) rf_gate_w<TK, R, KIND_SUM, 0>(wave, tile, U, lane);
      else rf_gate_w<TK, R, KIND_SUM, 1>(wave, tile, U, lane);
    } else {
      if (a.o[gi] == 0) rf_gate_w<TK, R, KIND_DIFF, 0>(wave, tile, U, lane);
      else rf_gate_w<TK, R, KIND_DIFF, 1>(wave, tile, U, lane);
    }
    if (more) rf_tab_put(tab[(gi + 1) & 1], 1, r);
    __syncthreads();
  }
  rf_gstore<TK, R>(dst + gb, a.sa, tile);
}

template <int TK>
__global__ __launch_bounds__(kBlock) void k_rfuse_adj(float *__restrict__ phi, float *__restrict__ lam, RFuseArgs a) {
  constexpr int R = kRFuseRAdj;
  using T = RTile<TK, R>;
  __shared__ __align__(16) float tp[T::SIZE];
  __shared__ __align__(16) float tl[T::SIZE];
  __shared__ float tab[2][2 * kTabN];
  __shared__ double red[kRFuseMax][4];  // per gate and wave: sums of lambda . A phi
  const uint32_t t = (uint32_t)xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t gb = rf_tile_base<TK, R>(t, a);
  float r[kTabPer];
  {
    float4 vp[T::PER], vl[T::PER];
    rf_gload<TK, R>(phi + gb, a.sa, vp);
    rf_gload<TK, R>(lam + gb, a.sa, vl);
    rf_tab_fetch(a.U[a.ng - 1], a.A[a.ng - 1], 2, r);
    rf_lput<TK, R>(tp, a.sa, vp);
    rf_lput<TK, R>(tl, a.sa, vl);
    rf_tab_put(tab[(a.ng - 1) & 1], 2, r);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int gi = a.ng - 1; gi >= 0; --gi) {
    if (gi > 0) rf_tab_fetch(a.U[gi - 1], a.A[gi - 1], 2, r);
    const LdsTab U{tab[gi & 1]}, A{tab[gi & 1] + kTabN};
    float g;
    if (a.kind[gi] == KIND_SUM) {
      g = a.o[gi] == 0 ? rf_adj_w<TK, R, KIND_SUM, 0>(wave, tp, tl, U, A, lane)
                       : rf_adj_w<TK, R, KIND_SUM, 1>(wave, tp, tl, U, A, lane);
    } else {
      g = a.o[gi] == 0 ? rf_adj_w<TK, R, KIND_DIFF, 0>(wave, tp, tl, U, A, lane)
                       : rf_adj_w<TK, R, KIND_DIFF, 1>(wave, tp, tl, U, A, lane);
    }
    if (gi > 0) rf_tab_put(tab[(gi - 1) & 1], 2, r);
    const double sw = wave_sum_d((double)g);
    if (lane == 0) red[gi][wave] = sw;
    __syncthreads();  // this step's LDS writes before the next step reads them
  }
  if (threadIdx.x < a.ng) {
    const double *w = red[threadIdx.x];
    a.part[threadIdx.x][t] = (w[0] + w[1]) + (w[2] + w[3]);
  }
  rf_gstore<TK, R>(phi + gb, a.sa, tp);
  rf_gstore<TK, R>(lam + gb, a.sa, tl);
}

#undef RF_WAVES

int rfuse_kind(int a) { return a == 0 ? 0 : (a == 1 ? 1 : 2); }

int check_rfuse(const Geometry &g, int a, int ng, const RFuseOp *ops, const void *p0, const void *p1) {
  if (!real_fuse_supported(g))
    return set_error(FOCK_ERR_UNSUPPORTED, "fused real gates at L=%d, d=%d (%u amplitudes)", g.L, g.d, g.n_amp);
  if (a < 0 || a + 2 > real_fuse_top(g))
    return set_error(FOCK_ERR_ARG, "fused real gates on modes %d..%d (top mode %d)", a, a + 2, real_fuse_top(g));
  if (ng < 1 || ng > kRFuseMax) return set_error(FOCK_ERR_ARG, "fused run of %d gates (1..%d)", ng, kRFuseMax);
  for (int k = 0; k < ng; ++k)
    if ((ops[k].kind != KIND_SUM && ops[k].kind != KIND_DIFF) || (ops[k].o != 0 && ops[k].o != 1) || !ops[k].U)
      return set_error(FOCK_ERR_ARG, "fused real gate %d: kind %d, offset %d", k, ops[k].kind, ops[k].o);
  if ((((uintptr_t)p0) | ((uintptr_t)p1)) & 15) return set_error(FOCK_ERR_ARG, "fused real gates: unaligned state");
  return FOCK_OK;
}

RFuseArgs rfuse_args(int a, int R, int ng, const RFuseOp *ops) {
  RFuseArgs r;
  memset(&r, 0, sizeof(r));
  r.sa = 1;
  for (int k = 0; k < a; ++k) r.sa *= (uint32_t)kRD;
  r.lo_tiles = r.sa >= (uint32_t)R ? r.sa / (uint32_t)R : 1u;
  r.ng = ng;
  for (int k = 0; k < ng; ++k) {
    r.kind[k] = ops[k].kind;
    r.o[k] = ops[k].o;
    r.U[k] = ops[k].U;
    r.A[k] = ops[k].A;
    r.part[k] = ops[k].part;
  }
  return r;
}

}  // namespace

bool real_fuse_supported(const Geometry &g) {
  return g.d == kRD && g.L >= 3 && g.L <= 10 && g.n_amp >= (1u << 21) && g.n_amp % (512u * kRFuseR) == 0;
}

int real_fuse_top(const Geometry &g) { return g.half ? g.L - 2 : g.L - 1; }

int real_fuse_blocks(const Geometry &g, bool reverse) {
  return (int)(g.n_amp / (512u * (uint32_t)(reverse ? kRFuseRAdj : kRFuseR)));
}

int launch_rfuse(const Geometry &g, int a, int ng, const RFuseOp *ops, const float *src, float *dst, hipStream_t s) {
  int rc = check_rfuse(g, a, ng, ops, src, dst);
  if (rc) return rc;
  const RFuseArgs ra = rfuse_args(a, kRFuseR, ng, ops);
  const int G = real_fuse_blocks(g, false);
  switch (rfuse_kind(a)) {
    case 0: hipLaunchKernelGGL(k_rfuse<0>, dim3(G), dim3(kBlock), 0, s, src, dst, ra); break;
    case 1: hipLaunchKernelGGL(k_rfuse<1>, dim3(G), dim3(kBlock), 0, s, src, dst, ra); break;
    default: hipLaunchKernelGGL(k_rfuse<2>, dim3(G), dim3(kBlock), 0, s, src, dst, ra); break;
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_rfuse_adj(const Geometry &g, int a, int ng, const RFuseOp *ops, float *phi, float *lam, hipStream_t s) {
  int rc = check_rfuse(g, a, ng, ops, phi, lam);
  if (rc) return rc;
  for (int k = 0; k < ng; ++k)
    if (!ops[k].A || !ops[k].part) return set_error(FOCK_ERR_ARG, "fused real reverse step %d: no A or partials", k);
  const RFuseArgs ra = rfuse_args(a, kRFuseRAdj, ng, ops);
  const int G = real_fuse_blocks(g, true);
  switch (rfuse_kind(a)) {
    case 0: hipLaunchKernelGGL(k_rfuse_adj<0>, dim3(G), dim3(kBlock), 0, s, phi, lam, ra); break;
    case 1: hipLaunchKernelGGL(k_rfuse_adj<1>, dim3(G), dim3(kBlock), 0, s, phi, lam, ra); break;
    default: hipLaunchKernelGGL(k_rfuse_adj<2>, dim3(G), dim3(kBlock), 0, s, phi, lam, ra); break;
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
