// Fused gate groups: descriptors, planning and launchers.
#pragma once

#include <vector>

#include "device_common.h"

namespace fock {

constexpr int kMaxFuseModes = 6;  // tile modes (d^s <= 4096 amplitudes)
constexpr int kMaxFuseGates = 8;  // gates per group

struct FuseGate {
  int type, kind;
  int ki, kj;  // tile positions of the gate's modes (kj = -1: single-mode gate on ki)
  int u_off;   // offset of the gate's table in the gate-table block
  int k;       // index of the gate in the circuit (row of its gradient partials)
};

struct FuseArgs {
  int s, nc, ng, ntile;
  uint32_t tstride[kMaxFuseModes];  // d^m of the tile modes, ascending (tile position 0 = mode 0)
  uint32_t cstride[kMaxL];          // d^m of the other modes, ascending (digits of the tile index)
  int boff[2 * kMaxD];              // offset of block s in a packed two-mode table
  const float2 *A[kTwoModeTypes];   // packed generator blocks of the two-mode types by table_slot (gradients)
  FuseGate g[kMaxFuseGates];
};

// A run of consecutive gates [k0, k1); s = 0 marks a single gate run by the
// per-gate kernels, otherwise the tile modes m[0..s).
// Gates k0..k1 of a circuit run together: an LDS tile over the modes m[0..s)
// (gate fusion, s > 0), a run of single-mode phase gates applied as one
// diagonal pass (diag), or one gate on its own kernel.
struct GateGroup {
  int k0, k1, s;
  int m[kMaxFuseModes];
  bool diag = false;
};

// Greedy grouping of a circuit (see plan_gate_groups in api.cpp).
bool fuse_supported(int d);
int fuse_max_modes(int L, int d);
int launch_fuse_fwd(int d, const FuseArgs &a, const float2 *src, float2 *dst, const float2 *utab, hipStream_t s);
int launch_fuse_adj(int d, const FuseArgs &a, float2 *phi, float2 *lam, const float2 *utab, double *partial, int rs,
                    hipStream_t s);

}  // namespace fock
