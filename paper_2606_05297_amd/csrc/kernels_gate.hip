// Two-mode gates exp(theta A) on a mode pair (i, j), their fused reverse
// (adjoint) step, single-mode diagonal gates, and the device-side gate build.
//
// A gate acts on each "fiber" (the d x d amplitudes over (n_i, n_j) for fixed
// other digits) block by block: number-conserving generators (HR, HI, DH)
// only mix states of equal n_i + n_j, two-mode squeezers (PR, PI) only states
// of equal n_i - n_j.  One thread owns one fiber; consecutive threads own
// fibers that differ in the lowest free mode, so every member load and store of
// a wavefront is a contiguous run when i >= 1.
//
// Reverse step (one reverse sweep for all dE/dtheta_k): with phi = phi_k and
// lam = lambda_k, accumulate Re <lam| A phi> over the fiber, then apply
// O_k^+ = exp(-theta A) to both phi and lam.  A is block diagonal with the
// same blocks, so the gradient term is fiber-local and fused with the update.
#include "device_common.h"

namespace fock {

struct GateLaunch {
  uint32_t nfib, si, sj;
  FastDiv dsi, dm1;
};

__device__ __forceinline__ uint32_t fiber_base(uint32_t f, const GateLaunch &g, int D) {
  const uint32_t t = fdiv(f, g.dsi);
  const uint32_t low = f - t * g.si;
  const uint32_t high = fdiv(t, g.dm1);
  const uint32_t mid = t - high * g.dm1.v;
  return low + mid * g.si * (uint32_t)D + high * g.sj * (uint32_t)D;
}

__device__ __forceinline__ void cmac(float2 &o, float2 u, float2 v) {
  o.x = fmaf(u.x, v.x, fmaf(-u.y, v.y, o.x));
  o.y = fmaf(u.x, v.y, fmaf(u.y, v.x, o.y));
}
// o += conj(u) * v
__device__ __forceinline__ void cmac_conj(float2 &o, float2 u, float2 v) {
  o.x = fmaf(u.x, v.x, fmaf(u.y, v.y, o.x));
  o.y = fmaf(u.x, v.y, fmaf(-u.y, v.x, o.y));
}

template <int D, int KIND, bool DAG>
__global__ __launch_bounds__(kBlock) void k_gate2(float2 *__restrict__ psi, const float2 *__restrict__ U, GateLaunch g) {
  const uint32_t f = (uint32_t)xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (f >= g.nfib) return;
  const uint32_t base = fiber_base(f, g, D);
  int off = 0;
#pragma unroll
  for (int s = 0; s <= 2 * D - 2; ++s) {
    const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
    float2 in[D];
#pragma unroll
    for (int q = 0; q < D; ++q)
      if (q < b) {
        const int a = lo + q;
        in[q] = psi[base + (uint32_t)a * g.si + (uint32_t)blk_nj(KIND, D, s, a) * g.sj];
      }
#pragma unroll
    for (int p = 0; p < D; ++p)
      if (p < b) {
        float2 o = make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 0; q < D; ++q)
          if (q < b) {
            if (DAG) cmac_conj(o, U[off + q * b + p], in[q]);
            else cmac(o, U[off + p * b + q], in[q]);
          }
        const int a = lo + p;
        psi[base + (uint32_t)a * g.si + (uint32_t)blk_nj(KIND, D, s, a) * g.sj] = o;
      }
    off += b * b;
  }
}

template <int D, int KIND>
__global__ __launch_bounds__(kBlock) void k_gate2_adj(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                      const float2 *__restrict__ U, const float2 *__restrict__ A,
                                                      double *__restrict__ partial, GateLaunch g) {
  __shared__ double red[4];
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t f = (uint32_t)vb * kBlock + threadIdx.x;
  float gacc = 0.f;
  if (f < g.nfib) {
    const uint32_t base = fiber_base(f, g, D);
    int off = 0;
#pragma unroll
    for (int s = 0; s <= 2 * D - 2; ++s) {
      const int lo = blk_lo(KIND, D, s), b = blk_hi(KIND, D, s) - lo + 1;
      float2 pv[D], lv[D];
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q < b) {
          const int a = lo + q;
          const uint32_t idx = base + (uint32_t)a * g.si + (uint32_t)blk_nj(KIND, D, s, a) * g.sj;
          pv[q] = phi[idx];
          lv[q] = lam[idx];
        }
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 ap = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) cmac(ap, A[off + p * b + q], pv[q]);
          gacc = fmaf(lv[p].x, ap.x, fmaf(lv[p].y, ap.y, gacc));
        }
#pragma unroll
      for (int p = 0; p < D; ++p)
        if (p < b) {
          float2 np = make_float2(0.f, 0.f), nl = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q < b) {
              const float2 u = U[off + q * b + p];
              cmac_conj(np, u, pv[q]);
              cmac_conj(nl, u, lv[q]);
            }
          const int a = lo + p;
          const uint32_t idx = base + (uint32_t)a * g.si + (uint32_t)blk_nj(KIND, D, s, a) * g.sj;
          phi[idx] = np;
          lam[idx] = nl;
        }
      off += b * b;
    }
  }
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

// ---------------------------------------------------------------- single-mode diagonal gates
// O = exp(theta A) with A = i f(N_r) is diag(exp(i theta f(n_r))); f = n^2 (KERR) or n (ROT).
struct DiagLaunch {
  int nrows, r, kerr;
  FastDiv dsr;  // divide a row index by d^(r-1) (r >= 1)
};

template <int D, bool DAG>
__global__ __launch_bounds__(kBlock) void k_diag(float2 *__restrict__ psi, const float2 *__restrict__ phg, DiagLaunch a) {
  __shared__ float2 ph[kMaxD];
  if (threadIdx.x < D) {
    const float2 p = phg[threadIdx.x];
    ph[threadIdx.x] = DAG ? make_float2(p.x, -p.y) : p;
  }
  __syncthreads();
  const int row = xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (row >= a.nrows) return;
  float2 v[D];
  load_row<D>(psi + (size_t)row * D, v);
  const int n = a.r == 0 ? 0 : (int)(fdiv((uint32_t)row, a.dsr) % D);
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const float2 p = ph[a.r == 0 ? q : n];
    float2 o = make_float2(0.f, 0.f);
    cmac(o, p, v[q]);
    v[q] = o;
  }
  store_row<D>(psi + (size_t)row * D, v);
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_diag_adj(float2 *__restrict__ phi, float2 *__restrict__ lam,
                                                     const float2 *__restrict__ phg, double *__restrict__ partial,
                                                     DiagLaunch a) {
  __shared__ float2 ph[kMaxD];
  __shared__ double red[4];
  if (threadIdx.x < D) ph[threadIdx.x] = phg[threadIdx.x];
  __syncthreads();
  const int vb = xcd_remap(blockIdx.x, gridDim.x);
  const int row = vb * kBlock + threadIdx.x;
  float gacc = 0.f;
  if (row < a.nrows) {
    float2 pv[D], lv[D];
    load_row<D>(phi + (size_t)row * D, pv);
    load_row<D>(lam + (size_t)row * D, lv);
    const int n = a.r == 0 ? 0 : (int)(fdiv((uint32_t)row, a.dsr) % D);
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const int lev = a.r == 0 ? q : n;
      const float f = a.kerr ? (float)(lev * lev) : (float)lev;
      // Re(conj(lam) * i f phi) = -f Im(conj(lam) phi)
      gacc = fmaf(-f, lv[q].x * pv[q].y - lv[q].y * pv[q].x, gacc);
      const float2 p = ph[lev];
      float2 np = make_float2(0.f, 0.f), nl = make_float2(0.f, 0.f);
      cmac_conj(np, p, pv[q]);
      cmac_conj(nl, p, lv[q]);
      pv[q] = np;
      lv[q] = nl;
    }
    store_row<D>(phi + (size_t)row * D, pv);
    store_row<D>(lam + (size_t)row * D, lv);
  }
  const double sg = block_sum_d((double)gacc, red);
  if (threadIdx.x == 0) partial[vb] = sg;
}

// ---------------------------------------------------------------- device-side gate build
// U = V diag(exp(i theta lambda)) V^+ per conserved block, from the FP64
// eigendata of G = -i A (A = i G), computed once per (type, d) on the host.
__global__ __launch_bounds__(kBlock) void k_gate_build(const double *__restrict__ theta,
                                                       const GateRec *__restrict__ recs, int n, EigTables T,
                                                       float2 *__restrict__ utab) {
  const int k = blockIdx.y;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const GateRec r = recs[k];
  const double th = theta[k];
  const int d = T.d;
  if (r.type == FOCK_KERR || r.type == FOCK_ROT) {
    if (e < d) {
      const double f = r.type == FOCK_KERR ? (double)(e * e) : (double)e;
      double sn, cs;
      sincos(th * f, &sn, &cs);
      utab[r.u_off + e] = make_float2((float)cs, (float)sn);
    }
    return;
  }
  if (e >= T.psize) return;
  int off = 0, loff = 0, b = 1;
  for (int s = 0; s <= 2 * d - 2; ++s) {
    b = blk_hi(KIND_SUM, d, s) - blk_lo(KIND_SUM, d, s) + 1;
    if (e < off + b * b) break;
    off += b * b;
    loff += b;
  }
  const int p = (e - off) / b, q = (e - off) % b;
  const double *V = T.V[r.type] + 2 * off;
  const double *lam = T.lam[r.type] + loff;
  double ur = 0.0, ui = 0.0;
  for (int m = 0; m < b; ++m) {
    double sn, cs;
    sincos(th * lam[m], &sn, &cs);
    const double pr = V[2 * (p * b + m)], pi = V[2 * (p * b + m) + 1];
    const double qr = V[2 * (q * b + m)], qi = V[2 * (q * b + m) + 1];
    // V[p][m] e^{i th lam} conj(V[q][m])
    const double tr = pr * cs - pi * sn, ti = pr * sn + pi * cs;
    ur += tr * qr + ti * qi;
    ui += ti * qr - tr * qi;
  }
  utab[r.u_off + e] = make_float2((float)ur, (float)ui);
}

int launch_gate_build(const double *theta, const GateRec *recs, int n, const EigTables &T, float2 *utab,
                      hipStream_t s) {
  if (n <= 0) return FOCK_OK;
  const int ex = (T.psize + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_gate_build, dim3(ex, n), dim3(kBlock), 0, s, theta, recs, n, T, utab);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

// ---------------------------------------------------------------- launchers
static GateLaunch make_gate_launch(const Geometry &g, int i, int j) {
  GateLaunch gl;
  uint32_t si = 1, sj = 1;
  for (int r = 0; r < i; ++r) si *= (uint32_t)g.d;
  for (int r = 0; r < j; ++r) sj *= (uint32_t)g.d;
  gl.si = si;
  gl.sj = sj;
  gl.nfib = g.n_amp / (uint32_t)(g.d * g.d);
  gl.dsi = make_fastdiv(si);
  gl.dm1 = make_fastdiv(sj / (si * (uint32_t)g.d));
  return gl;
}

int gate_blocks_count(const Geometry &g) {
  const uint32_t nf = g.n_amp / (uint32_t)(g.d * g.d);
  return (int)((nf + kBlock - 1) / kBlock);
}

template <int D>
static void launch_gate_d(const GateLaunch &gl, int kind, bool dag, const float2 *U, float2 *psi, int G,
                          hipStream_t s) {
  if (kind == KIND_SUM) {
    if (dag) hipLaunchKernelGGL((k_gate2<D, KIND_SUM, true>), dim3(G), dim3(kBlock), 0, s, psi, U, gl);
    else hipLaunchKernelGGL((k_gate2<D, KIND_SUM, false>), dim3(G), dim3(kBlock), 0, s, psi, U, gl);
  } else {
    if (dag) hipLaunchKernelGGL((k_gate2<D, KIND_DIFF, true>), dim3(G), dim3(kBlock), 0, s, psi, U, gl);
    else hipLaunchKernelGGL((k_gate2<D, KIND_DIFF, false>), dim3(G), dim3(kBlock), 0, s, psi, U, gl);
  }
}

#define FOCK_D_SWITCH(d, STMT)                                                                     \
  switch (d) {                                                                                     \
    case 2: { constexpr int D = 2; STMT; } break;                                                  \
    case 3: { constexpr int D = 3; STMT; } break;                                                  \
    case 4: { constexpr int D = 4; STMT; } break;                                                  \
    case 5: { constexpr int D = 5; STMT; } break;                                                  \
    case 6: { constexpr int D = 6; STMT; } break;                                                  \
    case 7: { constexpr int D = 7; STMT; } break;                                                  \
    case 8: { constexpr int D = 8; STMT; } break;                                                  \
    case 9: { constexpr int D = 9; STMT; } break;                                                  \
    case 10: { constexpr int D = 10; STMT; } break;                                                \
    case 11: { constexpr int D = 11; STMT; } break;                                                \
    case 12: { constexpr int D = 12; STMT; } break;                                                \
    case 13: { constexpr int D = 13; STMT; } break;                                                \
    case 14: { constexpr int D = 14; STMT; } break;                                                \
    case 15: { constexpr int D = 15; STMT; } break;                                                \
    case 16: { constexpr int D = 16; STMT; } break;                                                \
    default: return set_error(FOCK_ERR_UNSUPPORTED, "d=%d unsupported", d);                        \
  }

int launch_gate(const Geometry &g, int i, int j, int kind, bool dag, const float2 *U, float2 *psi,
                hipStream_t s) {
  const GateLaunch gl = make_gate_launch(g, i, j);
  const int G = gate_blocks_count(g);
  FOCK_D_SWITCH(g.d, launch_gate_d<D>(gl, kind, dag, U, psi, G, s));
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_gate_adj(const Geometry &g, int i, int j, int kind, const float2 *U, const float2 *A, float2 *phi,
                    float2 *lam, double *partial, hipStream_t s) {
  const GateLaunch gl = make_gate_launch(g, i, j);
  const int G = gate_blocks_count(g);
  if (kind == KIND_SUM) {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_gate2_adj<D, KIND_SUM>), dim3(G), dim3(kBlock), 0, s, phi, lam, U, A,
                                          partial, gl));
  } else {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_gate2_adj<D, KIND_DIFF>), dim3(G), dim3(kBlock), 0, s, phi, lam, U,
                                          A, partial, gl));
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int diag_blocks_count(const Geometry &g) {
  const uint32_t nrows = g.n_amp / (uint32_t)g.d;
  return (int)((nrows + kBlock - 1) / kBlock);
}

static DiagLaunch make_diag_launch(const Geometry &g, int r, int type) {
  DiagLaunch a;
  a.nrows = (int)(g.n_amp / (uint32_t)g.d);
  a.r = r;
  a.kerr = type == FOCK_KERR;
  uint32_t sr = 1;
  for (int k = 1; k < r; ++k) sr *= (uint32_t)g.d;
  a.dsr = make_fastdiv(sr);
  return a;
}

int launch_diag(const Geometry &g, int r, int type, bool dag, const float2 *ph, float2 *psi, hipStream_t s) {
  const DiagLaunch a = make_diag_launch(g, r, type);
  const int G = diag_blocks_count(g);
  if (dag) {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag<D, true>), dim3(G), dim3(kBlock), 0, s, psi, ph, a));
  } else {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag<D, false>), dim3(G), dim3(kBlock), 0, s, psi, ph, a));
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_diag_adj(const Geometry &g, int r, int type, const float2 *ph, float2 *phi, float2 *lam,
                    double *partial, hipStream_t s) {
  const DiagLaunch a = make_diag_launch(g, r, type);
  const int G = diag_blocks_count(g);
  FOCK_D_SWITCH(g.d, hipLaunchKernelGGL(k_diag_adj<D>, dim3(G), dim3(kBlock), 0, s, phi, lam, ph, partial, a));
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
