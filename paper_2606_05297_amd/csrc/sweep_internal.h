// Work items and launchers of the batched sweep kernels.
#pragma once

#include "gate_kernels.h"
#include "stencil_kernels.h"

namespace fock {

// Device pointer stored in an item list.  It is typed in the global address
// space: a kernel that reads a plain pointer from memory cannot tell where it
// points and emits flat memory instructions (64-bit address registers, waits
// shared with LDS traffic) for every access made through it.
template <class T>
struct GPtr {
  __attribute__((address_space(1))) T *p;
  GPtr() = default;
  __host__ __device__ GPtr(T *q) : p((__attribute__((address_space(1))) T *)q) {}
  __host__ __device__ operator T *() const { return (T *)p; }
};

// Read-only table pointer stored in an item list (gate matrices, generator
// blocks, pool descriptors): typed in the constant address space, so that
// wavefront-uniform reads through it become scalar loads, as they do through
// const __restrict__ kernel arguments.  The data must not change while a
// kernel that reads it runs.
template <class T>
struct CPtr {
  __attribute__((address_space(4))) T *p;
  CPtr() = default;
  __host__ __device__ CPtr(T *q) : p((__attribute__((address_space(4))) T *)q) {}
  __host__ __device__ operator T *() const { return (T *)p; }
};

// One workgroup's share of one gate (forward) or of its reverse step.
// variant: 0 = two-mode gate with i >= 1, 1 = two-mode gate on (0, j) (LDS),
// 2 = single-mode diagonal gate, 3 = a run of single-mode phase gates (run,
// tables from U on at the gate stride), 4 = two-mode gate on (0, j) at d = 8
// over several tiles (the single-point pipelined block).  Forward: dst <- O src.  Reverse:
// dst = phi, lam = lambda, partial[vb] <- Re<lam|A phi> of the workgroup (a
// run writes gate g's sum to partial[g * rs + vb]).
struct SweepItem {
  int p, vb, variant, kind, rs;
  GateLaunch gl;
  DiagLaunch dl;
  CPtr<const float2> U;
  CPtr<const float2> A;
  CPtr<const DiagRun> run;
  GPtr<const float2> src;
  GPtr<float2> dst;
  GPtr<float2> lam;
  GPtr<double> partial;
};
static_assert(sizeof(DiagRun) % 4 == 0, "run descriptors are copied word by word");

// One tile of H psi or of pool scoring for point p.
struct SweepHItem {
  int p, vb;
  GPtr<const float2> psi;
  GPtr<float2> hpsi;
  GPtr<double> partial;
};

// One fixed-order sum (see k_sweep_reduce).
struct SweepRItem {
  int p, mode, nblocks, ncols, col, stride;
  GPtr<const double> partial;
  GPtr<double> out;
};

struct SweepPoolArgs {
  PoolArgs args;
  CPtr<const PoolPair> pairs;
  CPtr<const PoolDiag> diags;
};

bool sweep_supports_d(int d);
int sweep_gate_blocks(int d, int namp, int i);
// Whether mode-0 items at this size run the pipelined multi-tile block (variant 4).
bool sweep_m0_piped(int d, int namp, int i);
// Whether the items of a gate layer at cutoff d are split into two classes
// (separate lists and launches): 0 = two-mode gates on modes i >= 1 and
// single-mode phases, 1 = two-mode gates on mode 0 (variant 1 items).  When
// not split, every item sits in the class-0 list and cls is ignored.
bool sweep_split_classes(int d);
int sweep_launch_gate(int d, int cls, const SweepItem *items, int n, const int *active, int grid, hipStream_t s);
int sweep_launch_adj(int d, int cls, const SweepItem *items, int n, const int *active, int grid, hipStream_t s);
int sweep_launch_h(int d, const SweepHItem *items, int n, const HamArgs *hams, const int *active, int grid,
                   hipStream_t s);
int sweep_launch_pool(int d, const SweepHItem *items, int n, const SweepPoolArgs *pa, const int *active, int grid,
                      hipStream_t s);
int sweep_launch_reduce(const SweepRItem *items, int n, const int *active, int grid, hipStream_t s);

// Host-side descriptors of the single-point launches (kernels_gate.hip).
GateLaunch gate_launch_params(const Geometry &g, int i, int j);
DiagLaunch diag_launch_params(const Geometry &g, int r, int type);

}  // namespace fock
