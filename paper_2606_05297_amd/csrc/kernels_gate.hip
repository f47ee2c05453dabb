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
#include <algorithm>
#include <cstring>

#include "gate_kernels.h"

namespace fock {

FOCK_GATE_EXTERN(2) FOCK_GATE_EXTERN(3) FOCK_GATE_EXTERN(4) FOCK_GATE_EXTERN(5) FOCK_GATE_EXTERN(6)
FOCK_GATE_EXTERN(7) FOCK_GATE_EXTERN(8) FOCK_GATE_EXTERN(9) FOCK_GATE_EXTERN(10) FOCK_GATE_EXTERN(11)
FOCK_GATE_EXTERN(12) FOCK_GATE_EXTERN(13) FOCK_GATE_EXTERN(14) FOCK_GATE_EXTERN(15) FOCK_GATE_EXTERN(16)

// ---------------------------------------------------------------- device-side gate build
// U = V diag(exp(i theta lambda)) V^+ per conserved block, from the FP64
// eigendata of G = -i A (A = i G), computed once per (type, d) on the host.
// Entry e of gate table r at angle th.
__device__ __forceinline__ void gate_build_entry(const GateRec &r, double th, int e, const EigTables &T,
                                                 float2 *__restrict__ utab) {
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
  if (r.type == FOCK_SR || r.type == FOCK_SI) {
    // dense d x d: U[p][q] = sum_m V[p][m] e^{i th lam_m} conj(V[q][m])
    if (e >= d * d) return;
    const int t = r.type == FOCK_SR ? 0 : 1;
    const int p = e / d, q = e % d;
    const double *V = T.V1[t];
    const double *lam = T.lam1[t];
    double ur = 0.0, ui = 0.0;
    for (int m = 0; m < d; ++m) {
      double sn, cs;
      sincos(th * lam[m], &sn, &cs);
      const double pr = V[2 * (p * d + m)], pi = V[2 * (p * d + m) + 1];
      const double qr = V[2 * (q * d + m)], qi = V[2 * (q * d + m) + 1];
      const double tr = pr * cs - pi * sn, ti = pr * sn + pi * cs;
      ur += tr * qr + ti * qi;
      ui += ti * qr - tr * qi;
    }
    utab[r.u_off + e] = make_float2((float)ur, (float)ui);
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
  const double *V = T.V[table_slot(r.type)] + 2 * off;
  const double *lam = T.lam[table_slot(r.type)] + loff;
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

__global__ __launch_bounds__(kBlock) void k_gate_build(const double *__restrict__ theta,
                                                       const GateRec *__restrict__ recs, int n, EigTables T,
                                                       float2 *__restrict__ utab) {
  const int k = blockIdx.y;
  if (k >= n) return;
  gate_build_entry(recs[k], theta[k], blockIdx.x * kBlock + threadIdx.x, T, utab);
}

// The same with the angles and records in the kernel arguments (no staging
// copy); workgroup (0, k) also stores gate k's record and angle for the
// kernels that read them later (the reduction of the reverse-step partials).
__global__ __launch_bounds__(kBlock) void k_gate_build_args(GateArgs ga, EigTables T, float2 *__restrict__ utab,
                                                            double *__restrict__ theta_out,
                                                            GateRec *__restrict__ recs_out) {
  const int k = blockIdx.y;
  if (k >= ga.n) return;
  const GateRec r = ga.rec[k];
  const double th = ga.theta[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    theta_out[k] = th;
    recs_out[k] = r;
  }
  gate_build_entry(r, th, blockIdx.x * kBlock + threadIdx.x, T, utab);
}

int launch_gate_build_args(const GateArgs &ga, const EigTables &T, float2 *utab, double *theta_out,
                           GateRec *recs_out, hipStream_t s) {
  if (ga.n <= 0) return FOCK_OK;
  if (ga.n > kArgGates) return set_error(FOCK_ERR_SIZE, "%d gates in the kernel arguments (at most %d)", ga.n, kArgGates);
  const int ex = (T.psize + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_gate_build_args, dim3(ex, ga.n), dim3(kBlock), 0, s, ga, T, utab, theta_out, recs_out);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
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

GateLaunch gate_launch_params(const Geometry &g, int i, int j) { return make_gate_launch(g, i, j); }

int gate_blocks_count(const Geometry &g, int i) {
  if (g.half && i == g.L - 2) return half_top_blocks(g);
  const uint32_t nf = g.n_amp / (uint32_t)(g.d * g.d);
  int fpb = 64;
  FOCK_D_SWITCH(g.d, fpb = launch_fibers_per_block_d<D>(i, nf));
  return (int)((nf + (uint32_t)fpb - 1) / (uint32_t)fpb);
}

int gate_blocks_max(const Geometry &g) {
  const int a = gate_blocks_count(g, 0), b = gate_blocks_count(g, 1);
  const int c = g.half ? gate_blocks_count(g, g.L - 2) : 0;
  return std::max(a, std::max(b, c));
}

int launch_gate(const Geometry &g, int i, int j, int kind, bool dag, const float2 *U, const float2 *src, float2 *psi,
                hipStream_t s) {
  if (g.half && j == g.L - 1) return launch_gate_half(g, i, j, kind, dag, U, src, psi, s);
  const GateLaunch gl = make_gate_launch(g, i, j);
  const int G = gate_blocks_count(g, i);
  FOCK_D_SWITCH(g.d, gate_launch_d<D>(gl, i, kind, dag, U, src, psi, G, s));
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_gate_adj(const Geometry &g, int i, int j, int kind, const float2 *U, const float2 *A, float2 *phi,
                    float2 *lam, double *partial, hipStream_t s, bool write_phi) {
  if (g.half && j == g.L - 1) return launch_gate_adj_half(g, i, j, kind, U, A, phi, lam, partial, s, write_phi);
  const GateLaunch gl = make_gate_launch(g, i, j);
  const int G = gate_blocks_count(g, i);
  FOCK_D_SWITCH(g.d, adj_launch_d<D>(gl, i, kind, U, A, phi, lam, partial, G, write_phi, s));
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

DiagLaunch diag_launch_params(const Geometry &g, int r, int type) { return make_diag_launch(g, r, type); }

int launch_diag(const Geometry &g, int r, int type, bool dag, const float2 *ph, const float2 *src, float2 *psi,
                hipStream_t s) {
  if (g.half) return set_error(FOCK_ERR_UNSUPPORTED, "phase gates in the parity-halved layout");
  const DiagLaunch a = make_diag_launch(g, r, type);
  const int G = diag_blocks_count(g);
  if (dag) {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag<D, true>), dim3(G), dim3(kBlock), 0, s, src, psi, ph, a));
  } else {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag<D, false>), dim3(G), dim3(kBlock), 0, s, src, psi, ph, a));
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_diag_adj(const Geometry &g, int r, int type, const float2 *ph, float2 *phi, float2 *lam,
                    double *partial, hipStream_t s, bool write_phi) {
  if (g.half) return set_error(FOCK_ERR_UNSUPPORTED, "phase gates in the parity-halved layout");
  const DiagLaunch a = make_diag_launch(g, r, type);
  const int G = diag_blocks_count(g);
  if (write_phi) {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag_adj<D, true>), dim3(G), dim3(kBlock), 0, s, phi, lam, ph, partial,
                                          a));
  } else {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag_adj<D, false>), dim3(G), dim3(kBlock), 0, s, phi, lam, ph, partial,
                                          a));
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

DiagRun diag_run_params(const Geometry &g, const fock_op_t *ops, int k0, int k1) {
  DiagRun a;
  memset(&a, 0, sizeof(a));
  a.nrows = (int)(g.n_amp / (uint32_t)g.d);
  a.ng = k1 - k0;
  a.stride = gate_stride(g.d);
  for (int q = 0; q < a.ng; ++q) {
    const fock_op_t &op = ops[k0 + q];
    a.r[q] = (int8_t)op.i;
    a.kerr[q] = (int8_t)(op.type == FOCK_KERR);
    uint32_t sr = 1;
    for (int k = 1; k < op.i; ++k) sr *= (uint32_t)g.d;
    a.dsr[q] = make_fastdiv(sr);
  }
  return a;
}

int launch_diag_run(const Geometry &g, const DiagRun &a, bool dag, const float2 *U, const float2 *src, float2 *psi,
                    hipStream_t s) {
  if (g.half) return set_error(FOCK_ERR_UNSUPPORTED, "phase gates in the parity-halved layout");
  if (a.ng < 1 || a.ng > kMaxDiagRun) return set_error(FOCK_ERR_ARG, "diagonal run of %d gates", a.ng);
  const int G = diag_blocks_count(g);
  if (dag) {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag_run<D, true>), dim3(G), dim3(kBlock), 0, s, src, psi, U, a));
  } else {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag_run<D, false>), dim3(G), dim3(kBlock), 0, s, src, psi, U, a));
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_diag_run_adj(const Geometry &g, const DiagRun &a, const float2 *U, float2 *phi, float2 *lam,
                        double *partial, int rs, hipStream_t s, bool write_phi) {
  if (g.half) return set_error(FOCK_ERR_UNSUPPORTED, "phase gates in the parity-halved layout");
  if (a.ng < 1 || a.ng > kMaxDiagRun) return set_error(FOCK_ERR_ARG, "diagonal run of %d gates", a.ng);
  const int G = diag_blocks_count(g);
  if (G > rs) return set_error(FOCK_ERR_SIZE, "diagonal run: %d partials per gate exceed the row stride %d", G, rs);
  if (write_phi) {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag_run_adj<D, true>), dim3(G), dim3(kBlock), 0, s, phi, lam, U,
                                          partial, rs, a));
  } else {
    FOCK_D_SWITCH(g.d, hipLaunchKernelGGL((k_diag_run_adj<D, false>), dim3(G), dim3(kBlock), 0, s, phi, lam, U,
                                          partial, rs, a));
  }
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
