// Two-pass H psi for chains of L = 8 modes with cutoff d = 8 (16,777,216
// amplitudes), open or ring.
//
// H (Sec. III, build sign convention):
//   H = sum_bonds [ -J (a_i^+ a_j + a_j^+ a_i) + Delta (a_i a_j + a_i^+ a_j^+) ]
//     + sum_r [ (U/2 + K) n_r (n_r - 1) - mu n_r ]
// with the truncated ladder action (Sec. II.A) on the flat index sum_r n_r 8^r:
//   (a_i^+ a_j psi)[n]   = dn(n_i) up(n_j) psi[n - e_i + e_j]
//   (a_j^+ a_i psi)[n]   = up(n_i) dn(n_j) psi[n + e_i - e_j]
//   (a_i a_j psi)[n]     = up(n_i) up(n_j) psi[n + e_i + e_j]
//   (a_i^+ a_j^+ psi)[n] = dn(n_i) dn(n_j) psi[n - e_i - e_j]
// where dn(m) = sqrt(m) and up(m) = sqrt(m + 1) for m < d - 1, up(d - 1) = 0:
// every term whose neighbour leaves the truncated space has coefficient 0, so
// its (wrapped, in-bounds) read is multiplied by zero.
//
// Why two passes.  Every one of the 8 modes is in a bond, so no tile that
// fits a CU's LDS holds all neighbours of its amplitudes; a one-pass kernel
// must gather most bond terms from L2 and other XCDs.  Here each pass keeps
// every neighbour it needs on chip:
//   column pass (first): bonds (4,5), (5,6), (6,7), the ring bond (0,7) and
//     the on-site terms of modes 4..7.  A workgroup owns a 16-amplitude chunk
//     of the low modes (a 128-byte segment at every high index) and streams
//     n7 = 0..7: slice k = all (n4, n5, n6) of the chunk at n7 = k (64 kB of
//     LDS).  Writes T = H_col psi into hpsi.
//   row pass (second): bonds (0,1), (1,2), (2,3), (3,4) and the on-site terms
//     of modes 0..3.  A workgroup owns a pencil (n5, n6, n7) and streams
//     n4 = 0..7: slice k = the contiguous 4096 amplitudes of modes 0..3 at
//     n4 = k (32 kB of LDS).  Reads T, writes H psi = T + H_row psi in place,
//     and the partials <psi|H psi> and <psi|psi> of its pencil.
// In both passes one mode lies in each thread's registers (n6 in the column
// pass, n3 in the row pass) and the streamed bond, (6,7) resp. (3,4), couples
// that mode with the streamed one: its terms are pushed from the thread's own
// registers of slice k into the accumulators of slices k - 1 and k + 1, with
// no LDS traffic.  Slice k - 1 is complete once slice k has been pushed and is
// written then.  Traffic: 8 B/amp read + 8 B/amp written (column pass),
// 16 B/amp read + 8 B/amp written (row pass), all in 128-byte or longer
// contiguous runs.
#include "device_common.h"

namespace fock {

namespace {

constexpr int kCols = 256;       // 16-amplitude chunks of the low modes 0..3
constexpr int kPencils = 512;    // (n5, n6, n7) pencils of the row pass
constexpr int kColThreads = 512;
constexpr int kRowThreads = 512;
constexpr int kS4 = 4096;        // stride of mode 4 (amplitudes)

// Row-pass pencils: (n5, n6, n7), or (n5, n6, m7) in the parity-halved layout.
__host__ __device__ inline int slab_pencils(const HamArgs &h) { return h.half ? kPencils / 2 : kPencils; }

__device__ __forceinline__ float dpp_from_left(float v) {  // lane i receives lane i - 1 (0 at a row start)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_from_right(float v) {  // lane i receives lane i + 1 (0 at a row end)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, true));
}

__device__ __forceinline__ void fma4(float4 &a, const float4 &v, float c) {
  a.x = fmaf(c, v.x, a.x);
  a.y = fmaf(c, v.y, a.y);
  a.z = fmaf(c, v.z, a.z);
  a.w = fmaf(c, v.w, a.w);
}
// a += v with factor c_lo on the first amplitude (x, y) and c_hi on the second (z, w)
__device__ __forceinline__ void fma4s(float4 &a, const float4 &v, float c_lo, float c_hi) {
  a.x = fmaf(c_lo, v.x, a.x);
  a.y = fmaf(c_lo, v.y, a.y);
  a.z = fmaf(c_hi, v.z, a.z);
  a.w = fmaf(c_hi, v.w, a.w);
}
__device__ __forceinline__ void fma2(float2 &a, const float2 &v, float c) {
  a.x = fmaf(c, v.x, a.x);
  a.y = fmaf(c, v.y, a.y);
}

// Real states: the column pass holds two real amplitudes per float2 (where the
// complex pass holds two complex ones per float4), the row pass one per float.
__device__ __forceinline__ void fma4(float2 &a, const float2 &v, float c) {
  a.x = fmaf(c, v.x, a.x);
  a.y = fmaf(c, v.y, a.y);
}
__device__ __forceinline__ void fma4s(float2 &a, const float2 &v, float c_lo, float c_hi) {
  a.x = fmaf(c_lo, v.x, a.x);
  a.y = fmaf(c_hi, v.y, a.y);
}
__device__ __forceinline__ void fma2(float &a, const float &v, float c) { a = fmaf(c, v, a); }
template <class V>
__device__ __forceinline__ V vzero();
template <>
__device__ __forceinline__ float4 vzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <>
__device__ __forceinline__ float2 vzero<float2>() { return make_float2(0.f, 0.f); }
template <>
__device__ __forceinline__ float vzero<float>() { return 0.f; }
__device__ __forceinline__ float2 vadd(const float2 &a, const float2 &b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float vadd(float a, float b) { return a + b; }
__device__ __forceinline__ float vdot(const float2 &a, const float2 &b) { return a.x * b.x + a.y * b.y; }
__device__ __forceinline__ float vdot(float a, float b) { return a * b; }
__device__ __forceinline__ float2 vdpp_left(const float2 &u) {
  return make_float2(dpp_from_left(u.x), dpp_from_left(u.y));
}
__device__ __forceinline__ float vdpp_left(float u) { return dpp_from_left(u); }
__device__ __forceinline__ float2 vdpp_right(const float2 &u) {
  return make_float2(dpp_from_right(u.x), dpp_from_right(u.y));
}
__device__ __forceinline__ float vdpp_right(float u) { return dpp_from_right(u); }

// Ladder factors: folded to constants where m is known at compile time (the
// unrolled register and stream indices), one square root per thread otherwise.
struct Coef {
  float J, Dl, c2, mu;
  __device__ __forceinline__ float dn(int m) const { return __builtin_sqrtf((float)m); }
  __device__ __forceinline__ float up(int m) const { return m < 7 ? __builtin_sqrtf((float)(m + 1)) : 0.f; }
  __device__ __forceinline__ float dg(int m) const { return c2 * (float)(m * (m - 1)) - mu * (float)m; }
};

__device__ __forceinline__ Coef make_coef(const HamArgs &h) {
  Coef c;
  c.J = h.J;
  c.Dl = h.Delta;
  c.c2 = h.c2;
  c.mu = h.mu;
  return c;
}

// Column pass.  Thread t: l = t & 7 (amplitudes 2l, 2l+1 of the chunk), n4 =
// (t >> 3) & 7, n5 = t >> 6; registers over n6.  A wavefront reads eight
// 128-byte segments per load (one per n4).
//
// HALF: the parity-halved layout, whose slices are m7 = 0..3 with n7 = 2 m7 + e
// and e = (n0 + .. + n6 + sigma) mod 2 per amplitude.  Bonds (4,5) and (5,6)
// keep the parity of n0..n6, so their neighbours sit in the same slice.  Bond
// (6,7) moves n6 by one, so e flips: an amplitude with e = 0 (n7 = 2 m7) reads
// its n7 + 1 neighbours in its own slice and its n7 - 1 neighbours in slice
// m7 - 1; one with e = 1 reads n7 - 1 in its own slice and n7 + 1 in slice
// m7 + 1.  e is fixed per (thread, register parity, float4 half), so each
// push carries a per-lane factor that selects the terms of the right parity.
// V = float4 (two complex amplitudes per lane) or float2 (two real ones, real
// states: same indexing, half the bytes; open chains only).
template <bool RING, bool HALF, class V = float4>
__global__ __launch_bounds__(kColThreads) void k_h8_col(const V *__restrict__ psi, V *__restrict__ tout, HamArgs h) {
  static_assert(!(RING && HALF), "the parity-halved layout is for open chains");
  static_assert(!(RING && sizeof(V) != sizeof(float4)), "real states: open chains");
  constexpr int NS = HALF ? 4 : 8;  // streamed slices
  __shared__ V sl[4096];  // [n6][n5][n4][l]
  const Coef C = make_coef(h);
  const int b = blockIdx.x;
  const int j = (b & 7) * (kCols / 8) + (b >> 3);  // XCD x takes chunks 32x .. 32x+31 (contiguous low-mode run)
  const int t = threadIdx.x;
  const int l = t & 7, n4 = (t >> 3) & 7, n5 = t >> 6;
  constexpr int S6 = kS4 / 2 * 64, S7 = kS4 / 2 * 512;  // float4 strides of modes 6, 7
  const size_t base = (size_t)(8 * j + l) + (size_t)(kS4 / 2) * (n4 + 8 * n5);
  const V *src = psi + base;
  V *dst = tout + base;
  // bond (4,5) coefficients and LDS offsets (wrapped indices carry weight 0)
  const float cA = -C.J * C.dn(n4) * C.up(n5), cB = -C.J * C.up(n4) * C.dn(n5);
  const float cC = C.Dl * C.up(n4) * C.up(n5), cD = C.Dl * C.dn(n4) * C.dn(n5);
  auto li = [&](int a4, int a5, int a6) { return (((a6 * 8) + (a5 & 7)) * 8 + (a4 & 7)) * 8 + l; };
  const int oA = li(n4 - 1, n5 + 1, 0), oB = li(n4 + 1, n5 - 1, 0), oC = li(n4 + 1, n5 + 1, 0),
            oD = li(n4 - 1, n5 - 1, 0);
  const int om = li(n4, n5 - 1, 0), op = li(n4, n5 + 1, 0);
  const float hm = -C.J * C.dn(n5), pm = C.Dl * C.dn(n5);  // (5,6) with the n5 - 1 column
  const float hp = -C.J * C.up(n5), pp = C.Dl * C.up(n5);  // (5,6) with the n5 + 1 column
  const float dg45 = C.dg(n4) + C.dg(n5);
  // ring bond (0,7): n0 of the two amplitudes
  const int q0 = 2 * (l & 3), q1 = q0 + 1;
  // HALF: per-lane factors for q = (register parity) ^ (float4 half): the
  // amplitude has e = par ^ q.  fJ/fD weigh the in-slice (6,7) reads of n6 - 1
  // and n6 + 1 (-J and Delta swap roles between e = 0 and e = 1), w1 / w0 keep
  // only e = 1 (pushed into m7 - 1) resp. e = 0 (pushed into m7 + 1).
  float fJ[2] = {0.f, 0.f}, fD[2] = {0.f, 0.f}, w0[2] = {0.f, 0.f}, w1[2] = {0.f, 0.f};
  if constexpr (HALF) {
    const int par = (octal_digit_parity((uint32_t)(16 * j + 2 * l)) + n4 + n5 + h.sector) & 1;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const bool odd = (par ^ q) != 0;
      fJ[q] = odd ? C.Dl : -C.J;
      fD[q] = odd ? -C.J : C.Dl;
      w1[q] = odd ? 1.f : 0.f;
      w0[q] = odd ? 0.f : 1.f;
    }
  }

  V own[8], nxt[8];
  V acc[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) own[a] = src[(size_t)a * S6];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    V(&am)[8] = acc[(k + 2) % 3];  // slice k - 1
    V(&a0)[8] = acc[k % 3];        // slice k
    V(&ap)[8] = acc[(k + 1) % 3];  // slice k + 1
    if (k > 0) __syncthreads();
#pragma unroll
    for (int a = 0; a < 8; ++a) sl[li(n4, n5, a)] = own[a];
    if (k < NS - 1) {
#pragma unroll
      for (int a = 0; a < 8; ++a) nxt[a] = src[(size_t)a * S6 + (size_t)(k + 1) * S7];
    }
    __syncthreads();
    if (k == 0) {
#pragma unroll
      for (int a = 0; a < 8; ++a) a0[a] = vzero<V>();
    }
    // ring bond: neighbours along n0 inside the chunk come from lanes l - 1
    // (its second amplitude, 2l - 1) and l + 1 (its first, 2l + 2) of the same n4
    // bond (6,7) and the ring bond, pushed from slice k into k - 1 ...
    if (k > 0) {
      if constexpr (HALF) {
        // outputs with e = 1 of slice k - 1 (n7 = 2k - 1) read n7 + 1 = 2k here
        const float u = __builtin_sqrtf((float)(2 * k));
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int q = a & 1;
          if (a > 0) fma4s(am[a], own[a - 1], -C.J * C.dn(a) * u * w1[q], -C.J * C.dn(a) * u * w1[q ^ 1]);
          if (a < 7) fma4s(am[a], own[a + 1], C.Dl * C.up(a) * u * w1[q], C.Dl * C.up(a) * u * w1[q ^ 1]);
        }
      } else {
        const float u = C.up(k - 1);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          if (a > 0) fma4(am[a], own[a - 1], -C.J * C.dn(a) * u);  // a6^+ a7: reads (n6 - 1, n7 + 1)
          if (a < 7) fma4(am[a], own[a + 1], C.Dl * C.up(a) * u);  // a6 a7:   reads (n6 + 1, n7 + 1)
          if constexpr (RING) {
            // a0^+ a7 reads (n0 - 1, n7 + 1); a0 a7 reads (n0 + 1, n7 + 1)
            const float h0 = -C.J * C.dn(q0) * u, h1 = -C.J * C.dn(q1) * u;
            const float p0 = C.Dl * C.up(q0) * u, p1 = C.Dl * C.up(q1) * u;
            const float lz = dpp_from_left(own[a].z), lw = dpp_from_left(own[a].w);
            const float rx = dpp_from_right(own[a].x), ry = dpp_from_right(own[a].y);
            am[a].x = fmaf(h0, lz, fmaf(p0, own[a].z, am[a].x));
            am[a].y = fmaf(h0, lw, fmaf(p0, own[a].w, am[a].y));
            am[a].z = fmaf(h1, own[a].x, fmaf(p1, rx, am[a].z));
            am[a].w = fmaf(h1, own[a].y, fmaf(p1, ry, am[a].w));
          }
        }
      }
#pragma unroll
      for (int a = 0; a < 8; ++a) dst[(size_t)a * S6 + (size_t)(k - 1) * S7] = am[a];
    }
    // ... and into k + 1
    if (k < NS - 1) {
      if constexpr (HALF) {
        // outputs with e = 0 of slice k + 1 (n7 = 2k + 2) read n7 - 1 = 2k + 1 here
        const float dnx = __builtin_sqrtf((float)(2 * k + 2));
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int q = a & 1;
          ap[a] = vzero<V>();
          if (a < 7) fma4s(ap[a], own[a + 1], -C.J * C.up(a) * dnx * w0[q], -C.J * C.up(a) * dnx * w0[q ^ 1]);
          if (a > 0) fma4s(ap[a], own[a - 1], C.Dl * C.dn(a) * dnx * w0[q], C.Dl * C.dn(a) * dnx * w0[q ^ 1]);
        }
      } else {
        const float dnx = C.dn(k + 1);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          ap[a] = vzero<V>();
          if (a < 7) fma4(ap[a], own[a + 1], -C.J * C.up(a) * dnx);  // a7^+ a6: reads (n6 + 1, n7 - 1)
          if (a > 0) fma4(ap[a], own[a - 1], C.Dl * C.dn(a) * dnx);  // a6^+ a7^+: reads (n6 - 1, n7 - 1)
          if constexpr (RING) {
            // a7^+ a0 reads (n0 + 1, n7 - 1); a0^+ a7^+ reads (n0 - 1, n7 - 1)
            const float h0 = -C.J * C.up(q0) * dnx, h1 = -C.J * C.up(q1) * dnx;
            const float p0 = C.Dl * C.dn(q0) * dnx, p1 = C.Dl * C.dn(q1) * dnx;
            const float lz = dpp_from_left(own[a].z), lw = dpp_from_left(own[a].w);
            const float rx = dpp_from_right(own[a].x), ry = dpp_from_right(own[a].y);
            ap[a].x = fmaf(h0, own[a].z, fmaf(p0, lz, ap[a].x));
            ap[a].y = fmaf(h0, own[a].w, fmaf(p0, lw, ap[a].y));
            ap[a].z = fmaf(h1, rx, fmaf(p1, own[a].x, ap[a].z));
            ap[a].w = fmaf(h1, ry, fmaf(p1, own[a].y, ap[a].w));
          }
        }
      }
    }
    // in-slice terms of slice k: on-site, bond (4,5), bond (5,6) (and, HALF,
    // bond (6,7) within the slice: n7 = 2k reads 2k + 1 and n7 = 2k + 1 reads 2k)
    if constexpr (HALF) {
      const float r = __builtin_sqrtf((float)(2 * k + 1));
      const float dge = C.dg(2 * k), dgo = C.dg(2 * k + 1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int q = a & 1;
        const float dgl = dg45 + C.dg(a) + w0[q] * dge + w1[q] * dgo;
        const float dgh = dg45 + C.dg(a) + w0[q ^ 1] * dge + w1[q ^ 1] * dgo;
        fma4s(a0[a], own[a], dgl, dgh);
        if (a > 0) fma4s(a0[a], own[a - 1], C.dn(a) * r * fJ[q], C.dn(a) * r * fJ[q ^ 1]);
        if (a < 7) fma4s(a0[a], own[a + 1], C.up(a) * r * fD[q], C.up(a) * r * fD[q ^ 1]);
      }
    } else {
      const float dgk = dg45 + C.dg(k);
#pragma unroll
      for (int a = 0; a < 8; ++a) fma4(a0[a], own[a], dgk + C.dg(a));
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int o6 = a * 64 * 8;
      fma4(a0[a], sl[oA + o6], cA);
      fma4(a0[a], sl[oB + o6], cB);
      fma4(a0[a], sl[oC + o6], cC);
      fma4(a0[a], sl[oD + o6], cD);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const V vm = sl[om + a * 512], vp = sl[op + a * 512];
      if (a > 0) {  // outputs n6 = a - 1 read (n5 -+ 1, n6 + 1)
        fma4(a0[a - 1], vm, hm * C.up(a - 1));
        fma4(a0[a - 1], vp, pp * C.up(a - 1));
      }
      if (a < 7) {  // outputs n6 = a + 1 read (n5 +- 1, n6 - 1)
        fma4(a0[a + 1], vp, hp * C.dn(a + 1));
        fma4(a0[a + 1], vm, pm * C.dn(a + 1));
      }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (k < NS - 1) own[a] = nxt[a];
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) dst[(size_t)a * S6 + (size_t)(NS - 1) * S7] = acc[(NS - 1) % 3][a];
}

// Row pass.  Thread t: n0 = t & 7, n1 = (t >> 3) & 7, n2 = t >> 6; registers
// over n3.  A wavefront reads 512 contiguous bytes per load.
// E = float2 (complex amplitudes) or float (real states).
template <class E = float2>
__global__ __launch_bounds__(kRowThreads) void k_h8_row(const E *__restrict__ psi, E *__restrict__ hpsi,
                                                        double *__restrict__ partial, HamArgs h) {
  __shared__ E tile[4096];  // [n3][n2][n1][n0]
  __shared__ double red[2 * kRowThreads / 64];
  const Coef C = make_coef(h);
  const int b = blockIdx.x;
  const int p = (b & 7) * (gridDim.x / 8) + (b >> 3);  // XCD x takes the pencils with n7 (m7) = x (x/2)
  const int t = threadIdx.x;
  const int n0 = t & 7, n1 = (t >> 3) & 7, n2 = t >> 6;
  const size_t base = (size_t)t + (size_t)p * 8 * kS4;
  const E *src = psi + base;
  E *dst = hpsi + base;
  auto ti = [&](int a0, int a1, int a2, int a3) { return (a0 & 7) + 8 * (a1 & 7) + 64 * (a2 & 7) + 512 * a3; };
  // bond (0,1): rows n1 +- 1 at n0, shifted along n0 across lanes
  const int r01p = ti(n0, n1 + 1, n2, 0), r01m = ti(n0, n1 - 1, n2, 0);
  const float c01a = -C.J * C.dn(n0) * C.up(n1);  // a0^+ a1: reads (n0 - 1, n1 + 1)
  const float c01b = -C.J * C.up(n0) * C.dn(n1);  // a1^+ a0: reads (n0 + 1, n1 - 1)
  const float c01c = C.Dl * C.up(n0) * C.up(n1);  // a0 a1:   reads (n0 + 1, n1 + 1)
  const float c01d = C.Dl * C.dn(n0) * C.dn(n1);  // a0^+ a1^+: reads (n0 - 1, n1 - 1)
  // bond (1,2)
  const int o12a = ti(n0, n1 - 1, n2 + 1, 0), o12b = ti(n0, n1 + 1, n2 - 1, 0), o12c = ti(n0, n1 + 1, n2 + 1, 0),
            o12d = ti(n0, n1 - 1, n2 - 1, 0);
  const float c12a = -C.J * C.dn(n1) * C.up(n2), c12b = -C.J * C.up(n1) * C.dn(n2);
  const float c12c = C.Dl * C.up(n1) * C.up(n2), c12d = C.Dl * C.dn(n1) * C.dn(n2);
  // bond (2,3): columns n2 -+ 1 over n3
  const int o23m = ti(n0, n1, n2 - 1, 0), o23p = ti(n0, n1, n2 + 1, 0);
  const float hm = -C.J * C.dn(n2), pm = C.Dl * C.dn(n2);
  const float hp = -C.J * C.up(n2), pp = C.Dl * C.up(n2);
  const float dg012 = C.dg(n0) + C.dg(n1) + C.dg(n2);

  E own[8], nxt[8], prev[8], tv[8];
  E acc[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) own[a] = src[(size_t)a * 512];
  float e = 0.f, nn = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    E(&am)[8] = acc[(k + 2) % 3];
    E(&a0)[8] = acc[k % 3];
    E(&ap)[8] = acc[(k + 1) % 3];
    if (k > 0) __syncthreads();
#pragma unroll
    for (int a = 0; a < 8; ++a) tile[t + 512 * a] = own[a];
    if (k < 7) {
#pragma unroll
      for (int a = 0; a < 8; ++a) nxt[a] = src[(size_t)a * 512 + (size_t)(k + 1) * kS4];
    }
    if (k > 0) {
#pragma unroll
      for (int a = 0; a < 8; ++a) tv[a] = dst[(size_t)a * 512 + (size_t)(k - 1) * kS4];  // column-pass terms
    }
    __syncthreads();
    if (k == 0) {
#pragma unroll
      for (int a = 0; a < 8; ++a) a0[a] = vzero<E>();
    }
    if (k > 0) {  // bond (3,4) pushed from slice k into k - 1, then slice k - 1 is complete
      const float u = C.up(k - 1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (a > 0) fma2(am[a], own[a - 1], -C.J * C.dn(a) * u);  // a3^+ a4: reads (n3 - 1, n4 + 1)
        if (a < 7) fma2(am[a], own[a + 1], C.Dl * C.up(a) * u);  // a3 a4:   reads (n3 + 1, n4 + 1)
        const E hv = vadd(am[a], tv[a]);
        e += vdot(prev[a], hv);
        nn += vdot(prev[a], prev[a]);
        dst[(size_t)a * 512 + (size_t)(k - 1) * kS4] = hv;
      }
    }
    if (k < 7) {  // ... and into k + 1
      const float dnx = C.dn(k + 1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        ap[a] = vzero<E>();
        if (a < 7) fma2(ap[a], own[a + 1], -C.J * C.up(a) * dnx);  // a4^+ a3: reads (n3 + 1, n4 - 1)
        if (a > 0) fma2(ap[a], own[a - 1], C.Dl * C.dn(a) * dnx);  // a3^+ a4^+: reads (n3 - 1, n4 - 1)
      }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      fma2(a0[a], own[a], dg012 + C.dg(a));  // on-site terms of modes 0..3 (mode 4's: column pass)
      // bond (0,1)
      const E u = tile[r01p + 512 * a], v = tile[r01m + 512 * a];
      const E ul = vdpp_left(u), ur = vdpp_right(u), vl = vdpp_left(v), vr = vdpp_right(v);
      fma2(a0[a], ul, c01a);
      fma2(a0[a], vr, c01b);
      fma2(a0[a], ur, c01c);
      fma2(a0[a], vl, c01d);
      // bond (1,2)
      fma2(a0[a], tile[o12a + 512 * a], c12a);
      fma2(a0[a], tile[o12b + 512 * a], c12b);
      fma2(a0[a], tile[o12c + 512 * a], c12c);
      fma2(a0[a], tile[o12d + 512 * a], c12d);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {  // bond (2,3)
      const E vm = tile[o23m + 512 * a], vp = tile[o23p + 512 * a];
      if (a > 0) {
        fma2(a0[a - 1], vm, hm * C.up(a - 1));
        fma2(a0[a - 1], vp, pp * C.up(a - 1));
      }
      if (a < 7) {
        fma2(a0[a + 1], vp, hp * C.dn(a + 1));
        fma2(a0[a + 1], vm, pm * C.dn(a + 1));
      }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      prev[a] = own[a];
      if (k < 7) own[a] = nxt[a];
    }
  }
  {
    E(&am)[8] = acc[7 % 3];
#pragma unroll
    for (int a = 0; a < 8; ++a) tv[a] = dst[(size_t)a * 512 + (size_t)7 * kS4];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const E hv = vadd(am[a], tv[a]);
      e += vdot(prev[a], hv);
      nn += vdot(prev[a], prev[a]);
      dst[(size_t)a * 512 + (size_t)7 * kS4] = hv;
    }
  }
  const double se = wave_sum_d((double)e), sn = wave_sum_d((double)nn);
  if ((t & 63) == 0) {
    red[2 * (t >> 6)] = se;
    red[2 * (t >> 6) + 1] = sn;
  }
  __syncthreads();
  if (t == 0) {
    double r0 = 0.0, r1 = 0.0;
#pragma unroll
    for (int w = 0; w < kRowThreads / 64; ++w) {
      r0 += red[2 * w];
      r1 += red[2 * w + 1];
    }
    partial[2 * p] = r0;
    partial[2 * p + 1] = r1;
  }
}

// ---------------------------------------------------------------- pool scoring
//
// Eq. (grad), g_k = 2 Re <H psi | A_k psi>, on the same two slab shapes: the
// row shape scores the pairs (0,1), (1,2), (2,3), (3,4) and every diagonal
// entry (KERR, ROT, CK), the column shape the pairs (4,5), (5,6), (6,7) and
// the ring pair (0,7).  For a pair (i, j) the four ladder neighbours of psi,
//   u1 = dn(n_i) up(n_j) psi[n - e_i + e_j]   (a_i^+ a_j)
//   u2 = up(n_i) dn(n_j) psi[n + e_i - e_j]   (a_j^+ a_i)
//   w1 = up(n_i) up(n_j) psi[n + e_i + e_j]   (a_i a_j)
//   w2 = dn(n_i) dn(n_j) psi[n - e_i - e_j]   (a_i^+ a_j^+)
// give (with c = conj(h[n]) x, h = H psi)
//   HR: Re(c(u1) - c(u2)),  HI: -Im(c(u1) + c(u2)),  DH: -Im(n_i c(u1) + (n_i + 1) c(u2)),
//   PR: Re(c(w1) - c(w2)),  PI: -Im(c(w1) + c(w2)),
// summed over n and doubled; a diagonal generator i f(N) gives -2 f(n) Im(conj(h) psi).
// Only psi needs neighbours (LDS slice and registers); H psi is read at each
// thread's own amplitudes.  The streamed pair's terms couple slice k with
// k - 1: at step k the thread pairs its own H psi of slice k with its psi of
// slice k - 1 and its H psi of slice k - 1 with its psi of slice k.

struct PairSums {  // per-thread sums of one pair, one per generator type
  float hr = 0.f, hi = 0.f, dh = 0.f, pr = 0.f, pi = 0.f;
};

// Accumulate one amplitude's four neighbour terms (already multiplied by their
// ladder factors) against h; ni = n_i of the amplitude.
__device__ __forceinline__ void pair_terms(PairSums &S, const float2 &h, const float2 &u1, const float2 &u2,
                                           const float2 &w1, const float2 &w2, float ni, bool X, bool Y, bool Dh) {
  if (X || Dh) {
    const float r1 = h.x * u1.x + h.y * u1.y, i1 = h.x * u1.y - h.y * u1.x;
    const float r2 = h.x * u2.x + h.y * u2.y, i2 = h.x * u2.y - h.y * u2.x;
    if (X) {
      S.hr += r1 - r2;
      S.hi -= i1 + i2;
    }
    if (Dh) S.dh -= ni * i1 + (ni + 1.f) * i2;
  }
  if (Y) {
    const float r1 = h.x * w1.x + h.y * w1.y, i1 = h.x * w1.y - h.y * w1.x;
    const float r2 = h.x * w2.x + h.y * w2.y, i2 = h.x * w2.y - h.y * w2.x;
    S.pr += r1 - r2;
    S.pi -= i1 + i2;
  }
}

__device__ __forceinline__ float2 cmul(float c, float2 v) { return make_float2(c * v.x, c * v.y); }
__device__ __forceinline__ float2 lo2(const float4 &v) { return make_float2(v.x, v.y); }
__device__ __forceinline__ float2 hi2(const float4 &v) { return make_float2(v.z, v.w); }

__device__ __forceinline__ bool want_x(const SlabPool &sp, int p) {
  return sp.slot[p][FOCK_HR] >= 0 || sp.slot[p][FOCK_HI] >= 0;
}
__device__ __forceinline__ bool want_y(const SlabPool &sp, int p) {
  return sp.slot[p][FOCK_PR] >= 0 || sp.slot[p][FOCK_PI] >= 0;
}
__device__ __forceinline__ bool want_d(const SlabPool &sp, int p) { return sp.slot[p][FOCK_DH] >= 0; }
__device__ __forceinline__ bool want_any(const SlabPool &sp, int p) {
  return want_x(sp, p) || want_y(sp, p) || want_d(sp, p);
}

// Diagonal entries on the row shape.  Each f(n) (KERR n_r^2, ROT n_r, CK
// n_r n_r2) is a polynomial of degree <= 2 in the register mode n3 whose
// coefficients depend only on the other modes, so with the slice sums
// m0 = sum_a Im(conj(h) psi), m1 = sum_a a Im(..), m2 = sum_a a^2 Im(..) over
// n3 = a each entry costs three products.  nv[r] is the thread's n_r (r != 3).
__device__ __forceinline__ void diag_slice(float *dsum, const SlabPool &sp, const float (&nv)[8], float m0, float m1,
                                           float m2) {
#pragma unroll
  for (int q = 0; q < kSlabDiag; ++q) {
    if (q >= sp.ndiag) break;
    const PoolDiag dq = sp.diag[q];
    const float vr = nv[dq.r & 7], vr2 = nv[dq.r2 & 7];
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
    if (dq.type == FOCK_KERR) {
      if (dq.r == 3) c2 = 1.f; else c0 = vr * vr;
    } else if (dq.type == FOCK_ROT) {
      if (dq.r == 3) c1 = 1.f; else c0 = vr;
    } else {  // CK on (r, r2), r != r2
      if (dq.r == 3) c1 = vr2; else if (dq.r2 == 3) c1 = vr; else c0 = vr * vr2;
    }
    dsum[q] -= c0 * m0 + c1 * m1 + c2 * m2;
  }
}

// Block reduction of per-thread slot values: red[w][slot] per wavefront (FP64
// over the lanes), then one FP64 partial per slot in a fixed order.
template <int NT>
__device__ __forceinline__ void slot_add(double (*red)[kMaxSlots], int slot, float v) {
  if (slot < 0) return;
  const double s = wave_sum_d((double)v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][slot] += s;
}
__device__ __forceinline__ void pair_slots(double (*red)[kMaxSlots], const SlabPool &sp, int p, const PairSums &S) {
  slot_add<0>(red, sp.slot[p][FOCK_HR], S.hr);
  slot_add<0>(red, sp.slot[p][FOCK_HI], S.hi);
  slot_add<0>(red, sp.slot[p][FOCK_DH], S.dh);
  slot_add<0>(red, sp.slot[p][FOCK_PR], S.pr);
  slot_add<0>(red, sp.slot[p][FOCK_PI], S.pi);
}
template <int NT>
__device__ __forceinline__ void write_slots(double (*red)[kMaxSlots], int nslots, double *__restrict__ out) {
  __syncthreads();
  for (int s = threadIdx.x; s < nslots; s += NT) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += red[w][s];
    out[s] = 2.0 * r;
  }
}

// Row shape: pencil (n5, n6, n7) streaming n4; thread (n0, n1, n2), registers n3.
__global__ __launch_bounds__(kRowThreads) void k_pool8_row(const float2 *__restrict__ psi,
                                                           const float2 *__restrict__ hpsi,
                                                           double *__restrict__ partial, SlabPool sp, HamArgs hcoef) {
  __shared__ float2 tile[4096];
  __shared__ double red[kRowThreads / 64][kMaxSlots];
  const int t = threadIdx.x;
  for (int e = t; e < (kRowThreads / 64) * kMaxSlots; e += kRowThreads) (&red[0][0])[e] = 0.0;
  const Coef C = make_coef(hcoef);
  const int b = blockIdx.x;
  const int p = (b & 7) * (gridDim.x / 8) + (b >> 3);
  const int n0 = t & 7, n1 = (t >> 3) & 7, n2 = t >> 6;
  const int n5 = p & 7, n6 = (p >> 3) & 7, n7 = p >> 6;
  const size_t base = (size_t)t + (size_t)p * 8 * kS4;
  auto ti = [&](int a0, int a1, int a2, int a3) { return (a0 & 7) + 8 * (a1 & 7) + 64 * (a2 & 7) + 512 * a3; };
  const bool on01 = want_any(sp, 0), on12 = want_any(sp, 1), on23 = want_any(sp, 2), on34 = want_any(sp, 3);
  PairSums S[4];
  float dsum[kSlabDiag];
#pragma unroll
  for (int q = 0; q < kSlabDiag; ++q) dsum[q] = 0.f;
  float2 own[8], prev[8], h[8], hp[8], nxt[8], hn[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    own[a] = psi[base + (size_t)a * 512];
    h[a] = hpsi[base + (size_t)a * 512];
  }
  __syncthreads();  // red cleared
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    if (k > 0) __syncthreads();
#pragma unroll
    for (int a = 0; a < 8; ++a) tile[t + 512 * a] = own[a];
    if (k < 7) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        nxt[a] = psi[base + (size_t)a * 512 + (size_t)(k + 1) * kS4];
        hn[a] = hpsi[base + (size_t)a * 512 + (size_t)(k + 1) * kS4];
      }
    }
    __syncthreads();
    if (on01) {
      const bool X = want_x(sp, 0), Y = want_y(sp, 0), Dh = want_d(sp, 0);
      const float ca = C.dn(n0) * C.up(n1), cb = C.up(n0) * C.dn(n1), cc = C.up(n0) * C.up(n1),
                  cd = C.dn(n0) * C.dn(n1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float2 u = tile[ti(n0, n1 + 1, n2, a)], v = tile[ti(n0, n1 - 1, n2, a)];
        const float2 ul = make_float2(dpp_from_left(u.x), dpp_from_left(u.y));
        const float2 ur = make_float2(dpp_from_right(u.x), dpp_from_right(u.y));
        const float2 vl = make_float2(dpp_from_left(v.x), dpp_from_left(v.y));
        const float2 vr = make_float2(dpp_from_right(v.x), dpp_from_right(v.y));
        pair_terms(S[0], h[a], cmul(ca, ul), cmul(cb, vr), cmul(cc, ur), cmul(cd, vl), (float)n0, X, Y, Dh);
      }
    }
    if (on12) {
      const bool X = want_x(sp, 1), Y = want_y(sp, 1), Dh = want_d(sp, 1);
      const float ca = C.dn(n1) * C.up(n2), cb = C.up(n1) * C.dn(n2), cc = C.up(n1) * C.up(n2),
                  cd = C.dn(n1) * C.dn(n2);
#pragma unroll
      for (int a = 0; a < 8; ++a)
        pair_terms(S[1], h[a], cmul(ca, tile[ti(n0, n1 - 1, n2 + 1, a)]), cmul(cb, tile[ti(n0, n1 + 1, n2 - 1, a)]),
                   cmul(cc, tile[ti(n0, n1 + 1, n2 + 1, a)]), cmul(cd, tile[ti(n0, n1 - 1, n2 - 1, a)]), (float)n1,
                   X, Y, Dh);
    }
    if (on23) {
      const bool X = want_x(sp, 2), Y = want_y(sp, 2), Dh = want_d(sp, 2);
      float2 vm[8], vp[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        vm[a] = tile[ti(n0, n1, n2 - 1, a)];
        vp[a] = tile[ti(n0, n1, n2 + 1, a)];
      }
      const float dm = C.dn(n2), um = C.up(n2);
      const float2 z = make_float2(0.f, 0.f);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float2 u1 = a < 7 ? cmul(dm * C.up(a), vm[a + 1]) : z;  // reads (n2 - 1, n3 + 1)
        const float2 u2 = a > 0 ? cmul(um * C.dn(a), vp[a - 1]) : z;  // reads (n2 + 1, n3 - 1)
        const float2 w1 = a < 7 ? cmul(um * C.up(a), vp[a + 1]) : z;  // reads (n2 + 1, n3 + 1)
        const float2 w2 = a > 0 ? cmul(dm * C.dn(a), vm[a - 1]) : z;  // reads (n2 - 1, n3 - 1)
        pair_terms(S[2], h[a], u1, u2, w1, w2, (float)n2, X, Y, Dh);
      }
    }
    if (on34 && k > 0) {
      const bool X = want_x(sp, 3), Y = want_y(sp, 3), Dh = want_d(sp, 3);
      const float2 z = make_float2(0.f, 0.f);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        // amplitudes of slice k read slice k - 1: a4^+ a3 (n3 + 1, n4 - 1), a3^+ a4^+ (n3 - 1, n4 - 1)
        const float2 u2 = a < 7 ? cmul(C.up(a) * C.dn(k), prev[a + 1]) : z;
        const float2 w2 = a > 0 ? cmul(C.dn(a) * C.dn(k), prev[a - 1]) : z;
        pair_terms(S[3], h[a], z, u2, z, w2, (float)a, X, Y, Dh);
        // amplitudes of slice k - 1 read slice k: a3^+ a4 (n3 - 1, n4 + 1), a3 a4 (n3 + 1, n4 + 1)
        const float2 u1 = a > 0 ? cmul(C.dn(a) * C.up(k - 1), own[a - 1]) : z;
        const float2 w1 = a < 7 ? cmul(C.up(a) * C.up(k - 1), own[a + 1]) : z;
        pair_terms(S[3], hp[a], u1, z, w1, z, (float)a, X, Y, Dh);
      }
    }
    // diagonal entries: -2 f(n) Im(conj(h) psi) (the factor 2 is applied at the end)
    if (sp.ndiag > 0) {
      float m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float im = h[a].x * own[a].y - h[a].y * own[a].x;
        m0 += im;
        m1 += (float)a * im;
        m2 += (float)(a * a) * im;
      }
      const float nv[8] = {(float)n0, (float)n1, (float)n2, 0.f, (float)k, (float)n5, (float)n6, (float)n7};
      diag_slice(dsum, sp, nv, m0, m1, m2);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      prev[a] = own[a];
      hp[a] = h[a];
      if (k < 7) {
        own[a] = nxt[a];
        h[a] = hn[a];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) pair_slots(red, sp, q, S[q]);
#pragma unroll
  for (int q = 0; q < kSlabDiag; ++q)
    if (q < sp.ndiag) slot_add<0>(red, sp.diag[q].slot, dsum[q]);
  write_slots<kRowThreads>(red, sp.nslots, partial + (size_t)p * sp.nslots);
}

// Column shape: chunk j streaming n7; thread (l, n4, n5) with amplitudes 2l,
// 2l + 1 of the chunk, registers n6.  The streamed pairs couple slices k and
// k + 1 through the prefetched slice k + 1 (psi and H psi), so no registers
// of slice k - 1 are kept.
//
// HALF (parity-halved layout, slices m7 with n7 = 2 m7 + e): for pair (6,7)
// an amplitude with e = 0 finds its n7 + 1 neighbours in its own slice and its
// n7 - 1 neighbours in slice m7 - 1; one with e = 1 finds n7 - 1 in its own
// slice and n7 + 1 in slice m7 + 1.  Step k scores the own-slice terms of
// slice k and the cross terms between slices k and k + 1 (e = 1 amplitudes of
// slice k, e = 0 amplitudes of slice k + 1); per-lane 0/1 factors pick them.
template <bool RING, bool HALF>
__global__ __launch_bounds__(kColThreads) void k_pool8_col(const float4 *__restrict__ psi,
                                                           const float4 *__restrict__ hpsi,
                                                           double *__restrict__ partial, SlabPool sp, HamArgs hcoef) {
  __shared__ float4 sl[4096];
  __shared__ double red[kColThreads / 64][kMaxSlots];
  const int t = threadIdx.x;
  for (int e = t; e < (kColThreads / 64) * kMaxSlots; e += kColThreads) (&red[0][0])[e] = 0.0;
  const Coef C = make_coef(hcoef);
  const int b = blockIdx.x;
  const int j = (b & 7) * (kCols / 8) + (b >> 3);
  const int l = t & 7, n4 = (t >> 3) & 7, n5 = t >> 6;
  constexpr int S6 = kS4 / 2 * 64, S7 = kS4 / 2 * 512;
  const size_t base = (size_t)(8 * j + l) + (size_t)(kS4 / 2) * (n4 + 8 * n5);
  auto li = [&](int a4, int a5, int a6) { return (((a6 * 8) + (a5 & 7)) * 8 + (a4 & 7)) * 8 + l; };
  const bool on45 = want_any(sp, 4), on56 = want_any(sp, 5), on67 = want_any(sp, 6), on07 = RING && want_any(sp, 7);
  const float q0 = (float)(2 * (l & 3)), q1 = q0 + 1.f;  // n0 of the two amplitudes
  const int iq0 = 2 * (l & 3), iq1 = iq0 + 1;
  const float2 z = make_float2(0.f, 0.f);
  static_assert(!(RING && HALF), "the parity-halved layout is for open chains");
  constexpr int NS = HALF ? 4 : 8;  // streamed slices
  float w0[2] = {0.f, 0.f}, w1[2] = {0.f, 0.f};  // HALF: e = par ^ q selects (q = register parity ^ half)
  if constexpr (HALF) {
    const int par = (octal_digit_parity((uint32_t)(16 * j + 2 * l)) + n4 + n5 + hcoef.sector) & 1;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      w1[q] = (par ^ q) ? 1.f : 0.f;
      w0[q] = 1.f - w1[q];
    }
  }
  PairSums S[4];
  float4 own[8], h[8], nxt[8], hn[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    own[a] = psi[base + (size_t)a * S6];
    h[a] = hpsi[base + (size_t)a * S6];
  }
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < NS; ++k) {
    if (k > 0) __syncthreads();
#pragma unroll
    for (int a = 0; a < 8; ++a) sl[li(n4, n5, a)] = own[a];
    if (k < NS - 1) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        nxt[a] = psi[base + (size_t)a * S6 + (size_t)(k + 1) * S7];
        hn[a] = hpsi[base + (size_t)a * S6 + (size_t)(k + 1) * S7];
      }
    }
    __syncthreads();
    if (on45) {
      const bool X = want_x(sp, 4), Y = want_y(sp, 4), Dh = want_d(sp, 4);
      const float ca = C.dn(n4) * C.up(n5), cb = C.up(n4) * C.dn(n5), cc = C.up(n4) * C.up(n5),
                  cd = C.dn(n4) * C.dn(n5);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float4 va = sl[li(n4 - 1, n5 + 1, a)], vb = sl[li(n4 + 1, n5 - 1, a)], vc = sl[li(n4 + 1, n5 + 1, a)],
                     vd = sl[li(n4 - 1, n5 - 1, a)];
        pair_terms(S[0], lo2(h[a]), cmul(ca, lo2(va)), cmul(cb, lo2(vb)), cmul(cc, lo2(vc)), cmul(cd, lo2(vd)),
                   (float)n4, X, Y, Dh);
        pair_terms(S[0], hi2(h[a]), cmul(ca, hi2(va)), cmul(cb, hi2(vb)), cmul(cc, hi2(vc)), cmul(cd, hi2(vd)),
                   (float)n4, X, Y, Dh);
      }
    }
    if (on56) {
      const bool X = want_x(sp, 5), Y = want_y(sp, 5), Dh = want_d(sp, 5);
      const float dm = C.dn(n5), um = C.up(n5);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float cu1 = a < 7 ? dm * C.up(a) : 0.f, cu2 = a > 0 ? um * C.dn(a) : 0.f;
        const float cw1 = a < 7 ? um * C.up(a) : 0.f, cw2 = a > 0 ? dm * C.dn(a) : 0.f;
        const float4 vmn = sl[li(n4, n5 - 1, a < 7 ? a + 1 : a)];  // (n5 - 1, n6 + 1)
        const float4 vpp = sl[li(n4, n5 + 1, a > 0 ? a - 1 : a)];  // (n5 + 1, n6 - 1)
        const float4 vpn = sl[li(n4, n5 + 1, a < 7 ? a + 1 : a)];  // (n5 + 1, n6 + 1)
        const float4 vmp = sl[li(n4, n5 - 1, a > 0 ? a - 1 : a)];  // (n5 - 1, n6 - 1)
        pair_terms(S[1], lo2(h[a]), cmul(cu1, lo2(vmn)), cmul(cu2, lo2(vpp)), cmul(cw1, lo2(vpn)),
                   cmul(cw2, lo2(vmp)), (float)n5, X, Y, Dh);
        pair_terms(S[1], hi2(h[a]), cmul(cu1, hi2(vmn)), cmul(cu2, hi2(vpp)), cmul(cw1, hi2(vpn)),
                   cmul(cw2, hi2(vmp)), (float)n5, X, Y, Dh);
      }
    }
    if (HALF && on67) {
      const bool X = want_x(sp, 6), Y = want_y(sp, 6), Dh = want_d(sp, 6);
      const float r = __builtin_sqrtf((float)(2 * k + 1)), rx = __builtin_sqrtf((float)(2 * k + 2));
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float2 ml = lo2(own[a > 0 ? a - 1 : a]), mh = hi2(own[a > 0 ? a - 1 : a]);  // n6 - 1
        const float2 pl = lo2(own[a < 7 ? a + 1 : a]), ph = hi2(own[a < 7 ? a + 1 : a]);  // n6 + 1
        const float dn = C.dn(a), up = C.up(a);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int q = (a & 1) ^ e;
          const float2 hv = e ? hi2(h[a]) : lo2(h[a]);
          const float2 vm = e ? mh : ml, vp = e ? ph : pl;
          // own slice: e = 0 reads (n6 -+ 1, n7 + 1) (u1, w1), e = 1 reads (n6 +- 1, n7 - 1) (u2, w2)
          pair_terms(S[2], hv, cmul(w0[q] * dn * r, vm), cmul(w1[q] * up * r, vp), cmul(w0[q] * up * r, vp),
                     cmul(w1[q] * dn * r, vm), (float)a, X, Y, Dh);
        }
      }
      if (k < NS - 1) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const float dn = C.dn(a), up = C.up(a);
          const float4 xm = nxt[a > 0 ? a - 1 : a], xp = nxt[a < 7 ? a + 1 : a];
          const float4 om = own[a > 0 ? a - 1 : a], op = own[a < 7 ? a + 1 : a];
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int q = (a & 1) ^ e;
            // e = 1 of slice k (n7 = 2k + 1) reads slice k + 1 at n7 + 1: a6^+ a7, a6 a7
            pair_terms(S[2], e ? hi2(h[a]) : lo2(h[a]), cmul(w1[q] * dn * rx, e ? hi2(xm) : lo2(xm)), z,
                       cmul(w1[q] * up * rx, e ? hi2(xp) : lo2(xp)), z, (float)a, X, Y, Dh);
            // e = 0 of slice k + 1 (n7 = 2k + 2) reads slice k at n7 - 1: a7^+ a6, a6^+ a7^+
            pair_terms(S[2], e ? hi2(hn[a]) : lo2(hn[a]), z, cmul(w0[q] * up * rx, e ? hi2(op) : lo2(op)), z,
                       cmul(w0[q] * dn * rx, e ? hi2(om) : lo2(om)), (float)a, X, Y, Dh);
          }
        }
      }
    }
    if (!HALF && on67 && k < 7) {
      const bool X = want_x(sp, 6), Y = want_y(sp, 6), Dh = want_d(sp, 6);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        // slice k reads slice k + 1: a6^+ a7 (n6 - 1, n7 + 1), a6 a7 (n6 + 1, n7 + 1)
        const float cu1 = a > 0 ? C.dn(a) * C.up(k) : 0.f, cw1 = a < 7 ? C.up(a) * C.up(k) : 0.f;
        const float4 xu = nxt[a > 0 ? a - 1 : a], xw = nxt[a < 7 ? a + 1 : a];
        pair_terms(S[2], lo2(h[a]), cmul(cu1, lo2(xu)), z, cmul(cw1, lo2(xw)), z, (float)a, X, Y, Dh);
        pair_terms(S[2], hi2(h[a]), cmul(cu1, hi2(xu)), z, cmul(cw1, hi2(xw)), z, (float)a, X, Y, Dh);
        // slice k + 1 reads slice k: a7^+ a6 (n6 + 1, n7 - 1), a6^+ a7^+ (n6 - 1, n7 - 1)
        const float cu2 = a < 7 ? C.up(a) * C.dn(k + 1) : 0.f, cw2 = a > 0 ? C.dn(a) * C.dn(k + 1) : 0.f;
        const float4 ou = own[a < 7 ? a + 1 : a], ow = own[a > 0 ? a - 1 : a];
        pair_terms(S[2], lo2(hn[a]), z, cmul(cu2, lo2(ou)), z, cmul(cw2, lo2(ow)), (float)a, X, Y, Dh);
        pair_terms(S[2], hi2(hn[a]), z, cmul(cu2, hi2(ou)), z, cmul(cw2, hi2(ow)), (float)a, X, Y, Dh);
      }
    }
    if (on07 && k < 7) {
      const bool X = want_x(sp, 7), Y = want_y(sp, 7), Dh = want_d(sp, 7);
      const float uk = C.up(k), dk = C.dn(k + 1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        // n0 -+ 1 inside the chunk: the thread's other amplitude or lanes l -+ 1 (weight 0 past n0 = 0, 7)
        const float2 xl = make_float2(dpp_from_left(nxt[a].z), dpp_from_left(nxt[a].w));
        const float2 xr = make_float2(dpp_from_right(nxt[a].x), dpp_from_right(nxt[a].y));
        const float2 ol = make_float2(dpp_from_left(own[a].z), dpp_from_left(own[a].w));
        const float2 orr = make_float2(dpp_from_right(own[a].x), dpp_from_right(own[a].y));
        // slice k reads slice k + 1: a0^+ a7 (n0 - 1, n7 + 1), a0 a7 (n0 + 1, n7 + 1)
        pair_terms(S[3], lo2(h[a]), cmul(C.dn(iq0) * uk, xl), z, cmul(C.up(iq0) * uk, hi2(nxt[a])), z, q0, X, Y,
                   Dh);
        pair_terms(S[3], hi2(h[a]), cmul(C.dn(iq1) * uk, lo2(nxt[a])), z, cmul(C.up(iq1) * uk, xr), z, q1, X, Y,
                   Dh);
        // slice k + 1 reads slice k: a7^+ a0 (n0 + 1, n7 - 1), a0^+ a7^+ (n0 - 1, n7 - 1)
        pair_terms(S[3], lo2(hn[a]), z, cmul(C.up(iq0) * dk, hi2(own[a])), z, cmul(C.dn(iq0) * dk, ol), q0, X, Y,
                   Dh);
        pair_terms(S[3], hi2(hn[a]), z, cmul(C.up(iq1) * dk, orr), z, cmul(C.dn(iq1) * dk, lo2(own[a])), q1, X, Y,
                   Dh);
      }
    }
    if (k < NS - 1) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        own[a] = nxt[a];
        h[a] = hn[a];
      }
    }
  }
#pragma unroll
  for (int p4 = 0; p4 < 4; ++p4) pair_slots(red, sp, 4 + p4, S[p4]);
  write_slots<kColThreads>(red, sp.nslots, partial + (size_t)(slab_pencils(hcoef) + j) * sp.nslots);
}

// Fused scoring, row shape: the row pass of H psi that also scores the pool
// entries of the row shape against the H psi it has just completed.  Two LDS
// slices: when slice s = k - 1 is finalised at step k (H psi(s) = column-pass
// terms + row terms), psi(s) is still in the other buffer, so the pairs
// (0,1), (1,2), (2,3) read their neighbours there; the streamed pair (3,4)
// reads psi(s +- 1) from the thread's registers (slices k and k - 2), and the
// diagonal entries use psi(s) itself.  Writes H psi, the energy/norm partials
// of its pencil and one partial per pool slot (the column shape's pairs are
// scored by k_pool8_col afterwards).
__global__ __launch_bounds__(kRowThreads) void k_h8_row_score(const float2 *__restrict__ psi,
                                                              float2 *__restrict__ hpsi,
                                                              double *__restrict__ partial,
                                                              double *__restrict__ ppart, SlabPool sp, HamArgs h) {
  __shared__ float2 tile[2][4096];  // psi of slices k (buffer k & 1) and k - 1
  __shared__ double red[kRowThreads / 64][kMaxSlots];
  __shared__ double red2[2 * kRowThreads / 64];
  const int t = threadIdx.x;
  for (int e = t; e < (kRowThreads / 64) * kMaxSlots; e += kRowThreads) (&red[0][0])[e] = 0.0;
  const Coef C = make_coef(h);
  const int b = blockIdx.x;
  const int p = (b & 7) * (gridDim.x / 8) + (b >> 3);
  const int n0 = t & 7, n1 = (t >> 3) & 7, n2 = t >> 6;
  const int n5 = p & 7, n6 = (p >> 3) & 7, n7 = p >> 6;
  const size_t base = (size_t)t + (size_t)p * 8 * kS4;
  const float2 *src = psi + base;
  float2 *dst = hpsi + base;
  auto ti = [&](int a0, int a1, int a2, int a3) { return (a0 & 7) + 8 * (a1 & 7) + 64 * (a2 & 7) + 512 * a3; };
  // H psi coefficients (as k_h8_row)
  const int r01p = ti(n0, n1 + 1, n2, 0), r01m = ti(n0, n1 - 1, n2, 0);
  const float c01a = C.dn(n0) * C.up(n1), c01b = C.up(n0) * C.dn(n1);
  const float c01c = C.up(n0) * C.up(n1), c01d = C.dn(n0) * C.dn(n1);
  const int o12a = ti(n0, n1 - 1, n2 + 1, 0), o12b = ti(n0, n1 + 1, n2 - 1, 0), o12c = ti(n0, n1 + 1, n2 + 1, 0),
            o12d = ti(n0, n1 - 1, n2 - 1, 0);
  const float c12a = C.dn(n1) * C.up(n2), c12b = C.up(n1) * C.dn(n2);
  const float c12c = C.up(n1) * C.up(n2), c12d = C.dn(n1) * C.dn(n2);
  const int o23m = ti(n0, n1, n2 - 1, 0), o23p = ti(n0, n1, n2 + 1, 0);
  const float dg012 = C.dg(n0) + C.dg(n1) + C.dg(n2);
  const bool on01 = want_any(sp, 0), on12 = want_any(sp, 1), on23 = want_any(sp, 2), on34 = want_any(sp, 3);
  PairSums S[4];
  float dsum[kSlabDiag];
#pragma unroll
  for (int q = 0; q < kSlabDiag; ++q) dsum[q] = 0.f;

  float2 own[8], nxt[8], prev[8], prev2[8], tv[8];
  // row-pass sums of slices k - 1 (am), k (a0) and k + 1 (ap), rotated each step
  float2 am[8], a0[8], ap[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) own[a] = src[(size_t)a * 512];
  float e = 0.f, nn = 0.f;
  // pool terms of slice s (its H psi in hf, psi(s) in prev, psi(s - 1) in prev2, psi(s + 1) in own)
  auto score = [&](int s, const float2 (&hf)[8], bool has_next) {
    const float2 *tl = tile[s & 1];
    const float2 z = make_float2(0.f, 0.f);
    if (on01) {
      const bool X = want_x(sp, 0), Y = want_y(sp, 0), Dh = want_d(sp, 0);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float2 u = tl[r01p + 512 * a], v = tl[r01m + 512 * a];
        const float2 ul = make_float2(dpp_from_left(u.x), dpp_from_left(u.y));
        const float2 ur = make_float2(dpp_from_right(u.x), dpp_from_right(u.y));
        const float2 vl = make_float2(dpp_from_left(v.x), dpp_from_left(v.y));
        const float2 vr = make_float2(dpp_from_right(v.x), dpp_from_right(v.y));
        pair_terms(S[0], hf[a], cmul(c01a, ul), cmul(c01b, vr), cmul(c01c, ur), cmul(c01d, vl), (float)n0, X, Y, Dh);
      }
    }
    if (on12) {
      const bool X = want_x(sp, 1), Y = want_y(sp, 1), Dh = want_d(sp, 1);
#pragma unroll
      for (int a = 0; a < 8; ++a)
        pair_terms(S[1], hf[a], cmul(c12a, tl[o12a + 512 * a]), cmul(c12b, tl[o12b + 512 * a]),
                   cmul(c12c, tl[o12c + 512 * a]), cmul(c12d, tl[o12d + 512 * a]), (float)n1, X, Y, Dh);
    }
    if (on23) {
      const bool X = want_x(sp, 2), Y = want_y(sp, 2), Dh = want_d(sp, 2);
      const float dm = C.dn(n2), um = C.up(n2);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float2 u1 = a < 7 ? cmul(dm * C.up(a), tl[o23m + 512 * (a + 1)]) : z;  // (n2 - 1, n3 + 1)
        const float2 u2 = a > 0 ? cmul(um * C.dn(a), tl[o23p + 512 * (a - 1)]) : z;  // (n2 + 1, n3 - 1)
        const float2 w1 = a < 7 ? cmul(um * C.up(a), tl[o23p + 512 * (a + 1)]) : z;  // (n2 + 1, n3 + 1)
        const float2 w2 = a > 0 ? cmul(dm * C.dn(a), tl[o23m + 512 * (a - 1)]) : z;  // (n2 - 1, n3 - 1)
        pair_terms(S[2], hf[a], u1, u2, w1, w2, (float)n2, X, Y, Dh);
      }
    }
    if (on34) {
      const bool X = want_x(sp, 3), Y = want_y(sp, 3), Dh = want_d(sp, 3);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        // slice s reads s + 1: a3^+ a4 (n3 - 1, n4 + 1), a3 a4 (n3 + 1, n4 + 1)
        const float2 u1 = (has_next && a > 0) ? cmul(C.dn(a) * C.up(s), own[a - 1]) : z;
        const float2 w1 = (has_next && a < 7) ? cmul(C.up(a) * C.up(s), own[a + 1]) : z;
        // slice s reads s - 1: a4^+ a3 (n3 + 1, n4 - 1), a3^+ a4^+ (n3 - 1, n4 - 1)
        const float2 u2 = (s > 0 && a < 7) ? cmul(C.up(a) * C.dn(s), prev2[a + 1]) : z;
        const float2 w2 = (s > 0 && a > 0) ? cmul(C.dn(a) * C.dn(s), prev2[a - 1]) : z;
        pair_terms(S[3], hf[a], u1, u2, w1, w2, (float)a, X, Y, Dh);
      }
    }
    if (sp.ndiag > 0) {
      float m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float im = hf[a].x * prev[a].y - hf[a].y * prev[a].x;
        m0 += im;
        m1 += (float)a * im;
        m2 += (float)(a * a) * im;
      }
      const float nv[8] = {(float)n0, (float)n1, (float)n2, 0.f, (float)s, (float)n5, (float)n6, (float)n7};
      diag_slice(dsum, sp, nv, m0, m1, m2);
    }
  };

  // Step k (0..8) stages slice k (k < 8), completes and scores slice k - 1
  // (k > 0) and adds the row terms of slice k.  Kept rolled: unrolled, the
  // kernel outgrows the instruction cache.
#pragma unroll
  for (int a = 0; a < 8; ++a) a0[a] = make_float2(0.f, 0.f);
#pragma unroll 1
  for (int k = 0; k <= 8; ++k) {
    if (k > 0) __syncthreads();
    if (k < 8) {
#pragma unroll
      for (int a = 0; a < 8; ++a) tile[k & 1][t + 512 * a] = own[a];
    }
    if (k < 7) {
#pragma unroll
      for (int a = 0; a < 8; ++a) nxt[a] = src[(size_t)a * 512 + (size_t)(k + 1) * kS4];
    }
    if (k > 0) {
#pragma unroll
      for (int a = 0; a < 8; ++a) tv[a] = dst[(size_t)a * 512 + (size_t)(k - 1) * kS4];
    }
    __syncthreads();
    if (k > 0) {  // bond (3,4) of slice k - 1 reading slice k; slice k - 1 complete: write, energy, scoring
      if (k < 8) {
        const float u = C.up(k - 1);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          if (a > 0) fma2(am[a], own[a - 1], -C.J * C.dn(a) * u);
          if (a < 7) fma2(am[a], own[a + 1], C.Dl * C.up(a) * u);
        }
      }
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        am[a] = make_float2(am[a].x + tv[a].x, am[a].y + tv[a].y);
        e += prev[a].x * am[a].x + prev[a].y * am[a].y;
        nn += prev[a].x * prev[a].x + prev[a].y * prev[a].y;
        dst[(size_t)a * 512 + (size_t)(k - 1) * kS4] = am[a];
      }
      score(k - 1, am, k < 8);
    }
    if (k == 8) break;
#pragma unroll
    for (int a = 0; a < 8; ++a) ap[a] = make_float2(0.f, 0.f);
    if (k < 7) {  // bond (3,4) of slice k + 1 reading slice k
      const float dnx = C.dn(k + 1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (a < 7) fma2(ap[a], own[a + 1], -C.J * C.up(a) * dnx);
        if (a > 0) fma2(ap[a], own[a - 1], C.Dl * C.dn(a) * dnx);
      }
    }
    const float2 *tl = tile[k & 1];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      fma2(a0[a], own[a], dg012 + C.dg(a));
      const float2 uu = tl[r01p + 512 * a], vv = tl[r01m + 512 * a];
      const float2 ul = make_float2(dpp_from_left(uu.x), dpp_from_left(uu.y));
      const float2 ur = make_float2(dpp_from_right(uu.x), dpp_from_right(uu.y));
      const float2 vl = make_float2(dpp_from_left(vv.x), dpp_from_left(vv.y));
      const float2 vr = make_float2(dpp_from_right(vv.x), dpp_from_right(vv.y));
      fma2(a0[a], ul, -C.J * c01a);
      fma2(a0[a], vr, -C.J * c01b);
      fma2(a0[a], ur, C.Dl * c01c);
      fma2(a0[a], vl, C.Dl * c01d);
      fma2(a0[a], tl[o12a + 512 * a], -C.J * c12a);
      fma2(a0[a], tl[o12b + 512 * a], -C.J * c12b);
      fma2(a0[a], tl[o12c + 512 * a], C.Dl * c12c);
      fma2(a0[a], tl[o12d + 512 * a], C.Dl * c12d);
    }
    {
      const float hm = -C.J * C.dn(n2), pm = C.Dl * C.dn(n2), hp = -C.J * C.up(n2), pp = C.Dl * C.up(n2);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const float2 vm = tl[o23m + 512 * a], vp = tl[o23p + 512 * a];
        if (a > 0) {
          fma2(a0[a - 1], vm, hm * C.up(a - 1));
          fma2(a0[a - 1], vp, pp * C.up(a - 1));
        }
        if (a < 7) {
          fma2(a0[a + 1], vp, hp * C.dn(a + 1));
          fma2(a0[a + 1], vm, pm * C.dn(a + 1));
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      prev2[a] = prev[a];
      prev[a] = own[a];
      if (k < 7) own[a] = nxt[a];
      am[a] = a0[a];
      a0[a] = ap[a];
    }
  }
  const double se = wave_sum_d((double)e), sn = wave_sum_d((double)nn);
  if ((t & 63) == 0) {
    red2[2 * (t >> 6)] = se;
    red2[2 * (t >> 6) + 1] = sn;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) pair_slots(red, sp, q, S[q]);
#pragma unroll
  for (int q = 0; q < kSlabDiag; ++q)
    if (q < sp.ndiag) slot_add<0>(red, sp.diag[q].slot, dsum[q]);
  __syncthreads();
  if (t == 0) {
    double r0 = 0.0, r1 = 0.0;
#pragma unroll
    for (int w = 0; w < kRowThreads / 64; ++w) {
      r0 += red2[2 * w];
      r1 += red2[2 * w + 1];
    }
    partial[2 * p] = r0;
    partial[2 * p + 1] = r1;
  }
  write_slots<kRowThreads>(red, sp.nslots, ppart + (size_t)p * sp.nslots);
}

}  // namespace

bool apply_h2_supported(const HamArgs &h) {
  return slab_stencil_ok(h.L, h.d) && (!h.half || (!h.periodic_wrap && (h.sector == 0 || h.sector == 1)));
}

// Partials written: 2 per pencil, columns (<psi|H psi>, <psi|psi>).
int apply_h2_blocks(const HamArgs &h) { return slab_pencils(h); }

static void launch_col(const HamArgs &h, const float2 *psi, float2 *hpsi, hipStream_t s) {
  if (h.half)
    hipLaunchKernelGGL((k_h8_col<false, true>), dim3(kCols), dim3(kColThreads), 0, s, (const float4 *)psi,
                       (float4 *)hpsi, h);
  else if (h.periodic_wrap)
    hipLaunchKernelGGL((k_h8_col<true, false>), dim3(kCols), dim3(kColThreads), 0, s, (const float4 *)psi,
                       (float4 *)hpsi, h);
  else
    hipLaunchKernelGGL((k_h8_col<false, false>), dim3(kCols), dim3(kColThreads), 0, s, (const float4 *)psi,
                       (float4 *)hpsi, h);
}

static void launch_pool_col(const SlabPool &sp, const HamArgs &h, const float2 *psi, const float2 *hpsi,
                            double *partial, hipStream_t s) {
  if (h.half)
    hipLaunchKernelGGL((k_pool8_col<false, true>), dim3(kCols), dim3(kColThreads), 0, s, (const float4 *)psi,
                       (const float4 *)hpsi, partial, sp, h);
  else if (h.periodic_wrap)
    hipLaunchKernelGGL((k_pool8_col<true, false>), dim3(kCols), dim3(kColThreads), 0, s, (const float4 *)psi,
                       (const float4 *)hpsi, partial, sp, h);
  else
    hipLaunchKernelGGL((k_pool8_col<false, false>), dim3(kCols), dim3(kColThreads), 0, s, (const float4 *)psi,
                       (const float4 *)hpsi, partial, sp, h);
}

int launch_apply_h2(const HamArgs &h, const float2 *psi, float2 *hpsi, double *partial, int *nblocks,
                    hipStream_t s) {
  if (!apply_h2_supported(h)) return set_error(FOCK_ERR_UNSUPPORTED, "two-pass H psi needs L = 8, d = 8");
  launch_col(h, psi, hpsi, s);
  hipLaunchKernelGGL((k_h8_row<float2>), dim3(slab_pencils(h)), dim3(kRowThreads), 0, s, psi, hpsi, partial, h);
  FOCK_HIP(hipGetLastError());
  *nblocks = apply_h2_blocks(h);
  return FOCK_OK;
}

bool apply_h2_real_supported(const HamArgs &h) { return apply_h2_supported(h) && !h.periodic_wrap; }

int launch_apply_h2_real(const HamArgs &h, const float *psi, float *hpsi, double *partial, int *nblocks,
                         hipStream_t s) {
  if (!apply_h2_real_supported(h))
    return set_error(FOCK_ERR_UNSUPPORTED, "two-pass H psi on real states needs an open L = 8, d = 8 chain");
  if (h.half)
    hipLaunchKernelGGL((k_h8_col<false, true, float2>), dim3(kCols), dim3(kColThreads), 0, s, (const float2 *)psi,
                       (float2 *)hpsi, h);
  else
    hipLaunchKernelGGL((k_h8_col<false, false, float2>), dim3(kCols), dim3(kColThreads), 0, s, (const float2 *)psi,
                       (float2 *)hpsi, h);
  hipLaunchKernelGGL((k_h8_row<float>), dim3(slab_pencils(h)), dim3(kRowThreads), 0, s, psi, hpsi, partial, h);
  FOCK_HIP(hipGetLastError());
  *nblocks = apply_h2_blocks(h);
  return FOCK_OK;
}

int pool_slab_blocks(const HamArgs &h) { return slab_pencils(h) + kCols; }

// The parity-halved layout has no stored n7, which the diagonal entries need.
static int check_slab_pool(const SlabPool &sp, const HamArgs &h) {
  if (sp.nslots < 1 || sp.nslots > kMaxSlots || sp.ndiag < 0 || sp.ndiag > kSlabDiag)
    return set_error(FOCK_ERR_ARG, "slab pool: %d slots, %d diagonal entries", sp.nslots, sp.ndiag);
  if (h.half && sp.ndiag > 0)
    return set_error(FOCK_ERR_UNSUPPORTED, "diagonal pool entries in the parity-halved layout");
  return FOCK_OK;
}

int launch_score_slab(const SlabPool &sp, const HamArgs &h, const float2 *psi, float2 *hpsi, double *hpart,
                      double *ppart, hipStream_t s) {
  if (!apply_h2_supported(h)) return set_error(FOCK_ERR_UNSUPPORTED, "fused scoring needs L = 8, d = 8");
  int rc = check_slab_pool(sp, h);
  if (rc) return rc;
  launch_col(h, psi, hpsi, s);
  hipLaunchKernelGGL(k_h8_row_score, dim3(slab_pencils(h)), dim3(kRowThreads), 0, s, psi, hpsi, hpart, ppart, sp,
                     h);
  launch_pool_col(sp, h, psi, hpsi, ppart, s);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_pool_slab(const SlabPool &sp, const HamArgs &h, const float2 *psi, const float2 *hpsi, double *partial,
                     int *nblocks, hipStream_t s) {
  if (!apply_h2_supported(h)) return set_error(FOCK_ERR_UNSUPPORTED, "slab pool scoring needs L = 8, d = 8");
  int rc = check_slab_pool(sp, h);
  if (rc) return rc;
  hipLaunchKernelGGL(k_pool8_row, dim3(slab_pencils(h)), dim3(kRowThreads), 0, s, psi, hpsi, partial, sp, h);
  launch_pool_col(sp, h, psi, hpsi, partial, s);
  FOCK_HIP(hipGetLastError());
  *nblocks = pool_slab_blocks(h);
  return FOCK_OK;
}

}  // namespace fock
