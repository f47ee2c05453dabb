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
__device__ __forceinline__ void fma2(float2 &a, const float2 &v, float c) {
  a.x = fmaf(c, v.x, a.x);
  a.y = fmaf(c, v.y, a.y);
}

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
template <bool RING>
__global__ __launch_bounds__(kColThreads) void k_h8_col(const float4 *__restrict__ psi, float4 *__restrict__ tout,
                                                         HamArgs h) {
  __shared__ float4 sl[4096];  // [n6][n5][n4][l]
  const Coef C = make_coef(h);
  const int b = blockIdx.x;
  const int j = (b & 7) * (kCols / 8) + (b >> 3);  // XCD x takes chunks 32x .. 32x+31 (contiguous low-mode run)
  const int t = threadIdx.x;
  const int l = t & 7, n4 = (t >> 3) & 7, n5 = t >> 6;
  constexpr int S6 = kS4 / 2 * 64, S7 = kS4 / 2 * 512;  // float4 strides of modes 6, 7
  const size_t base = (size_t)(8 * j + l) + (size_t)(kS4 / 2) * (n4 + 8 * n5);
  const float4 *src = psi + base;
  float4 *dst = tout + base;
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

  float4 own[8], nxt[8];
  float4 acc[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) own[a] = src[(size_t)a * S6];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    float4(&am)[8] = acc[(k + 2) % 3];  // slice k - 1
    float4(&a0)[8] = acc[k % 3];        // slice k
    float4(&ap)[8] = acc[(k + 1) % 3];  // slice k + 1
    if (k > 0) __syncthreads();
#pragma unroll
    for (int a = 0; a < 8; ++a) sl[li(n4, n5, a)] = own[a];
    if (k < 7) {
#pragma unroll
      for (int a = 0; a < 8; ++a) nxt[a] = src[(size_t)a * S6 + (size_t)(k + 1) * S7];
    }
    __syncthreads();
    if (k == 0) {
#pragma unroll
      for (int a = 0; a < 8; ++a) a0[a] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // ring bond: neighbours along n0 inside the chunk come from lanes l - 1
    // (its second amplitude, 2l - 1) and l + 1 (its first, 2l + 2) of the same n4
    // bond (6,7) and the ring bond, pushed from slice k into k - 1 ...
    if (k > 0) {
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
#pragma unroll
      for (int a = 0; a < 8; ++a) dst[(size_t)a * S6 + (size_t)(k - 1) * S7] = am[a];
    }
    // ... and into k + 1
    if (k < 7) {
      const float dnx = C.dn(k + 1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        ap[a] = make_float4(0.f, 0.f, 0.f, 0.f);
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
    // in-slice terms of slice k: on-site, bond (4,5), bond (5,6)
    const float dgk = dg45 + C.dg(k);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      fma4(a0[a], own[a], dgk + C.dg(a));
      const int o6 = a * 64 * 8;
      fma4(a0[a], sl[oA + o6], cA);
      fma4(a0[a], sl[oB + o6], cB);
      fma4(a0[a], sl[oC + o6], cC);
      fma4(a0[a], sl[oD + o6], cD);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const float4 vm = sl[om + a * 512], vp = sl[op + a * 512];
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
      if (k < 7) own[a] = nxt[a];
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) dst[(size_t)a * S6 + (size_t)7 * S7] = acc[7 % 3][a];
}

// Row pass.  Thread t: n0 = t & 7, n1 = (t >> 3) & 7, n2 = t >> 6; registers
// over n3.  A wavefront reads 512 contiguous bytes per load.
__global__ __launch_bounds__(kRowThreads) void k_h8_row(const float2 *__restrict__ psi, float2 *__restrict__ hpsi,
                                                        double *__restrict__ partial, HamArgs h) {
  __shared__ float2 tile[4096];  // [n3][n2][n1][n0]
  __shared__ double red[2 * kRowThreads / 64];
  const Coef C = make_coef(h);
  const int b = blockIdx.x;
  const int p = (b & 7) * (kPencils / 8) + (b >> 3);  // XCD x takes the pencils with n7 = x
  const int t = threadIdx.x;
  const int n0 = t & 7, n1 = (t >> 3) & 7, n2 = t >> 6;
  const size_t base = (size_t)t + (size_t)p * 8 * kS4;
  const float2 *src = psi + base;
  float2 *dst = hpsi + base;
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

  float2 own[8], nxt[8], prev[8], tv[8];
  float2 acc[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) own[a] = src[(size_t)a * 512];
  float e = 0.f, nn = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    float2(&am)[8] = acc[(k + 2) % 3];
    float2(&a0)[8] = acc[k % 3];
    float2(&ap)[8] = acc[(k + 1) % 3];
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
      for (int a = 0; a < 8; ++a) a0[a] = make_float2(0.f, 0.f);
    }
    if (k > 0) {  // bond (3,4) pushed from slice k into k - 1, then slice k - 1 is complete
      const float u = C.up(k - 1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (a > 0) fma2(am[a], own[a - 1], -C.J * C.dn(a) * u);  // a3^+ a4: reads (n3 - 1, n4 + 1)
        if (a < 7) fma2(am[a], own[a + 1], C.Dl * C.up(a) * u);  // a3 a4:   reads (n3 + 1, n4 + 1)
        const float2 hv = make_float2(am[a].x + tv[a].x, am[a].y + tv[a].y);
        e += prev[a].x * hv.x + prev[a].y * hv.y;
        nn += prev[a].x * prev[a].x + prev[a].y * prev[a].y;
        dst[(size_t)a * 512 + (size_t)(k - 1) * kS4] = hv;
      }
    }
    if (k < 7) {  // ... and into k + 1
      const float dnx = C.dn(k + 1);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        ap[a] = make_float2(0.f, 0.f);
        if (a < 7) fma2(ap[a], own[a + 1], -C.J * C.up(a) * dnx);  // a4^+ a3: reads (n3 + 1, n4 - 1)
        if (a > 0) fma2(ap[a], own[a - 1], C.Dl * C.dn(a) * dnx);  // a3^+ a4^+: reads (n3 - 1, n4 - 1)
      }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      fma2(a0[a], own[a], dg012 + C.dg(a));  // on-site terms of modes 0..3 (mode 4's: column pass)
      // bond (0,1)
      const float2 u = tile[r01p + 512 * a], v = tile[r01m + 512 * a];
      const float2 ul = make_float2(dpp_from_left(u.x), dpp_from_left(u.y));
      const float2 ur = make_float2(dpp_from_right(u.x), dpp_from_right(u.y));
      const float2 vl = make_float2(dpp_from_left(v.x), dpp_from_left(v.y));
      const float2 vr = make_float2(dpp_from_right(v.x), dpp_from_right(v.y));
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
      const float2 vm = tile[o23m + 512 * a], vp = tile[o23p + 512 * a];
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
    float2(&am)[8] = acc[7 % 3];
#pragma unroll
    for (int a = 0; a < 8; ++a) tv[a] = dst[(size_t)a * 512 + (size_t)7 * kS4];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const float2 hv = make_float2(am[a].x + tv[a].x, am[a].y + tv[a].y);
      e += prev[a].x * hv.x + prev[a].y * hv.y;
      nn += prev[a].x * prev[a].x + prev[a].y * prev[a].y;
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

}  // namespace

bool apply_h2_supported(const HamArgs &h) { return slab_stencil_ok(h.L, h.d); }

// Partials written: 2 * kPencils doubles, columns (<psi|H psi>, <psi|psi>) per pencil.
int apply_h2_blocks() { return kPencils; }

int launch_apply_h2(const HamArgs &h, const float2 *psi, float2 *hpsi, double *partial, int *nblocks,
                    hipStream_t s) {
  if (!apply_h2_supported(h)) return set_error(FOCK_ERR_UNSUPPORTED, "two-pass H psi needs L = 8, d = 8");
  if (h.periodic_wrap)
    hipLaunchKernelGGL(k_h8_col<true>, dim3(kCols), dim3(kColThreads), 0, s, (const float4 *)psi, (float4 *)hpsi, h);
  else
    hipLaunchKernelGGL(k_h8_col<false>, dim3(kCols), dim3(kColThreads), 0, s, (const float4 *)psi, (float4 *)hpsi, h);
  hipLaunchKernelGGL(k_h8_row, dim3(kPencils), dim3(kRowThreads), 0, s, psi, hpsi, partial, h);
  FOCK_HIP(hipGetLastError());
  *nblocks = apply_h2_blocks();
  return FOCK_OK;
}

}  // namespace fock
