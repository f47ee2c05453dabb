// Work items and launchers of the batched sweep kernels.
#pragma once

#include "gate_kernels.h"
#include "stencil_kernels.h"

namespace fock {

// One workgroup's share of one gate (forward) or of its reverse step.
// variant: 0 = two-mode gate with i >= 1, 1 = two-mode gate on (0, j) (LDS),
// 2 = single-mode diagonal gate.  Forward: dst <- O src.  Reverse: dst = phi,
// lam = lambda, partial[vb] <- Re<lam|A phi> of the workgroup.
struct SweepItem {
  int p, vb, variant, kind;
  GateLaunch gl;
  DiagLaunch dl;
  const float2 *U;
  const float2 *A;
  const float2 *src;
  float2 *dst;
  float2 *lam;
  double *partial;
};

// One tile of H psi or of pool scoring for point p.
struct SweepHItem {
  int p, vb;
  const float2 *psi;
  float2 *hpsi;
  double *partial;
};

// One fixed-order sum (see k_sweep_reduce).
struct SweepRItem {
  int p, mode, nblocks, ncols, col, stride;
  const double *partial;
  double *out;
};

struct SweepPoolArgs {
  PoolArgs args;
  const PoolPair *pairs;
  const PoolDiag *diags;
};

bool sweep_supports_d(int d);
int sweep_gate_blocks(int d, int namp, int i);
int sweep_launch_gate(int d, const SweepItem *items, int n, const int *active, int grid, hipStream_t s);
int sweep_launch_adj(int d, const SweepItem *items, int n, const int *active, int grid, hipStream_t s);
int sweep_launch_h(int d, const SweepHItem *items, int n, const HamArgs *hams, const int *active, int grid,
                   hipStream_t s);
int sweep_launch_pool(int d, const SweepHItem *items, int n, const SweepPoolArgs *pa, const int *active, int grid,
                      hipStream_t s);
int sweep_launch_reduce(const SweepRItem *items, int n, const int *active, int grid, hipStream_t s);

// Host-side descriptors of the single-point launches (kernels_gate.hip).
GateLaunch gate_launch_params(const Geometry &g, int i, int j);
DiagLaunch diag_launch_params(const Geometry &g, int r, int type);

}  // namespace fock
